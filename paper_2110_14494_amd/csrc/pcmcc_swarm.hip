// Batched uniform-field swarms (arXiv:2110.14494 Sec. 2.2.2): many
// independent electron swarms, each in its own field E/N and with its own
// size, advanced together by one persistent cooperative launch; their
// moments give flux and bulk transport coefficients (Sec. 2.2.2) with a
// temporal-growth model.
//
// Layout: swarm s owns a contiguous region of cap_s slots in each of two
// particle buffers.  A step runs the segment-pipelined mover (pcmcc_flight.hpp)
// over all swarms' electrons at once, the swarm index being the electron's
// group (its field, its random-number key, its destination region); survivors
// are appended to region s of the next buffer, one atomic per swarm and
// batch.  Newborns of all swarms share one queue that carries the swarm
// index.  Population control runs when an electron is loaded in the next
// step (keep with probability 2^-k, or duplicate).  Moments are summed
// exactly in 128-bit fixed point, so they do not depend on the order in
// which particles land in the buffers.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "pcmcc_device.hpp"
#include "pcmcc_flight.hpp"
#include "pcmcc_internal.hpp"
#include "pcmcc_mover.hpp"

namespace cg = cooperative_groups;

namespace pcmcc {

__device__ __forceinline__ Key swarm_key(Key k, int s) { return Key{k.k0, k.k1 ^ (uint32_t)s}; }

// Group policy of the mover for swarms: the group is the swarm index.
struct SwarmField {
  const double* az;    // LDS [S]: acceleration along z
  const float* a_abs;  // LDS [S]: |az| in single precision
  Key base;
  using Where = int;
  // The run's key passes through an empty asm statement at every use, so that
  // the Philox round keys of its uniform word are derived there with scalar
  // adds instead of being hoisted out of the mover loop (where they spill into
  // vector lanes and come back one v_readlane each).
  __device__ __forceinline__ Key key(uint32_t s) const {
    uint32_t k0 = base.k0, k1 = base.k1;
    asm volatile("" : "+s"(k0), "+s"(k1));
    return swarm_key(Key{k0, k1}, (int)s);
  }
  __device__ __forceinline__ double3 accel(double, double, double, uint32_t s, Where&) const {
    return make_double3(0.0, 0.0, az[s]);
  }
  __device__ __forceinline__ void bound_at(Where, uint32_t s, float, float, float& a, float& da) const {
    a = a_abs[s];
    da = 0.0f;
  }
};

// Swarm of global electron index g: the last s with prefix[s] <= g.
__device__ __forceinline__ int swarm_of(const uint32_t* prefix, int S, uint32_t g);

// Phase 1 source: the electrons of all swarms (prefix of counts in LDS),
// with the population control decided at the previous commit applied as
// they are loaded: keep with probability 2^-k, or duplicate (the duplicate
// joins the newborn queue and starts from t = 0).
struct SwarmLoad {
  KArg<Soa> cur;
  const uint64_t* base;
  const uint32_t* prefix;
  const int* pck;
  int n_swarms;
  Key key;
  uint32_t step;
  BirthSink dup;  // duplicates: the generation-0 newborn queue
  uint32_t* psteps;
  // The swarm of a chunk's first electron, found once when the wave takes the
  // chunk; an electron of the chunk walks forward from it (a chunk is at most
  // kChunkMax electrons, so it seldom crosses a swarm boundary).
  __device__ __forceinline__ uint32_t hint(uint64_t first) const {
    return (uint32_t)swarm_of(prefix, n_swarms, (uint32_t)first);
  }
  __device__ __forceinline__ void load(uint64_t g, Flight& f, uint32_t s0) const {
    int s = (int)s0;
    while (prefix[s + 1] <= (uint32_t)g) ++s;
    const uint64_t i = g - prefix[s];
    PState p;
    load_p(cur.get(), base[s] + i, p);
    const int k = pck[s];
    bool keep = true;
    if (k != 0) {
      const uint4 r = draw(swarm_key(key, s), p.id, step - 1, 0, TAG_AUX);
      if (k > 0) {
        keep = unif(r.x) < ldexpf(1.0f, -k);
      } else {
        PState d = p;
        d.id = (uint64_t)r.y | ((uint64_t)r.z << 32);
        BirthSink q = dup;
        q.tag = (uint32_t)s;
        q.push(d, 0.0f);
        (*psteps)++;
      }
    }
    if (!keep) return;
    (*psteps)++;
    flight_start(f, p, 0.0, 0u, (uint32_t)s);
  }
};

// Phase 2 source: the newborn queue (with swarm indices and birth times).
struct SwarmPend {
  KArg<PendSoa> qk;
  __device__ __forceinline__ uint32_t hint(uint64_t) const { return 0u; }
  __device__ __forceinline__ void load(uint64_t i, Flight& f, uint32_t) const {
    PState p;
    float tb;
    const PendSoa q = qk.get();
    load_pend(q, i, p, tb);
    flight_start(f, p, (double)tb, 0u, q.sw[i]);
  }
};

// Destination: survivors are appended to their swarm's region of the next
// buffer (staged per wave, one atomic per swarm and batch); attachments are
// counted per swarm.
struct SwarmPlace {
  KArg<Soa> nxt;
  const uint64_t* base;
  const uint64_t* cap_s;
  unsigned long long* n_nxt;
  unsigned long long* cum_att;
  unsigned* overflow;
  __device__ __forceinline__ bool can_open() const { return true; }
  __device__ __forceinline__ uint32_t open_chunk(uint64_t, uint32_t) const { return 0u; }
  __device__ __forceinline__ void tag(Flight&, uint32_t) const {}
  __device__ __forceinline__ uint32_t done_all(const Flight& f, bool parked, Cnt&, WaveStage* L,
                                               uint32_t n_staged) const {
    group_count(cum_att, f.tag, parked && f.seg == EV_ATTACHED);
    bool staged = false;
    if (parked && f.seg == EV_DONE) {
      const PState p = flight_record(f);
      const uint32_t s = n_staged + rank_in(__ballot(1));
      if (s < kStage) {
        L->s[0][s] = p.x;
        L->s[1][s] = p.y;
        L->s[2][s] = p.z;
        L->s[3][s] = p.vx;
        L->s[4][s] = p.vy;
        L->s[5][s] = p.vz;
        L->s[6][s] = p.w;
        L->stag[s] = f.tag;
        L->sid[s] = p.id;
        staged = true;
      } else {
        const uint64_t slot = atomicAdd(&n_nxt[f.tag], 1ull);
        if (slot < cap_s[f.tag])
          store_p(nxt.get(), base[f.tag] + slot, p);
        else
          atomicOr(overflow, OVF_CAPACITY);
      }
    }
    return n_staged + (uint32_t)__popcll(__ballot(staged));
  }
  __device__ __forceinline__ void flush(WaveStage* L, uint32_t n) const {
    const uint32_t l = lane_id();
    const bool mine = l < n;
    const uint32_t s = mine ? L->stag[l] : 0u;
    const uint64_t slot = group_reserve(n_nxt, s, mine);
    if (!mine) return;
    if (slot < cap_s[s]) {
      PState p;
      p.x = L->s[0][l];
      p.y = L->s[1][l];
      p.z = L->s[2][l];
      p.vx = L->s[3][l];
      p.vy = L->s[4][l];
      p.vz = L->s[5][l];
      p.w = L->s[6][l];
      p.id = L->sid[l];
      store_p(nxt.get(), base[s] + slot, p);
    } else {
      atomicOr(overflow, OVF_CAPACITY);
    }
  }
};

// 128-bit two's-complement accumulator word pair (lo, hi), exact and order
// independent: the carry out of the low word is added to the high word.
__device__ __forceinline__ void add128_atomic(unsigned long long* acc, unsigned long long lo, long long hi) {
  const unsigned long long old = atomicAdd(&acc[0], lo);
  if (old + lo < old) hi += 1;
  if (hi) atomicAdd(&acc[1], (unsigned long long)hi);
}

__device__ __forceinline__ void add128(unsigned long long& lo, long long& hi, long long v) {
  const unsigned long long l = (unsigned long long)v;
  const unsigned long long s = lo + l;
  hi += (v < 0 ? -1 : 0) + (s < lo ? 1 : 0);
  lo = s;
}

// Fixed-point exponents of the moments (value * 2^e, |value * 2^e| < 2^54 so
// that a 256-particle block sum fits in 64 bits).
constexpr int kMomExp[kNMom] = {0, 53, 53, 53, 53, 53, 25, 25, 25, 24, 24, 36, 0, 0};
constexpr double kMomLim[kNMom] = {2.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0x1p29, 0x1p29, 0x1p29, 0x1p30, 0x1p30,
                                    0x1p18, 0x1p53, 0x1p53};

// Block-level exclusive scan of per-swarm tile counts into LDS prefix[0..S].
__device__ void tile_prefix(const unsigned long long* n, int S, int tile, uint32_t* prefix, uint32_t* tmp) {
  const int T = blockDim.x;
  const int per = (S + T - 1) / T;
  const int lo = threadIdx.x * per, hi = min(lo + per, S);
  uint32_t sum = 0;
  for (int s = lo; s < hi; ++s) sum += (uint32_t)((ld_acq(&n[s]) + tile - 1) / tile);
  tmp[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < T; off <<= 1) {
    const uint32_t v = threadIdx.x >= (unsigned)off ? tmp[threadIdx.x - off] : 0u;
    __syncthreads();
    tmp[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? tmp[threadIdx.x - 1] : 0u;
  for (int s = lo; s < hi; ++s) {
    prefix[s] = run;
    run += (uint32_t)((ld_acq(&n[s]) + tile - 1) / tile);
  }
  if (threadIdx.x == T - 1) prefix[S] = tmp[T - 1];
  __syncthreads();
}

__device__ __forceinline__ int swarm_of(const uint32_t* prefix, int S, uint32_t g) {
  int lo = 0, hi = S;  // prefix[lo] <= g < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Swarm owning tile tt: the last s with prefix[s] <= tt.
__device__ __forceinline__ int find_swarm(const uint32_t* prefix, int S, uint32_t tt) {
  int lo = 0, hi = S;  // prefix[lo] <= tt < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= tt)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// ---------------------------------------------------------------------------
template <int BS, int REFILL, int ROW>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(4))) void k_swarm_steps(SwarmArgs A) {
  extern __shared__ float smem[];
  cg::grid_group grid = cg::this_grid();
  const Tab T = stage_tables(A.T, A.S, smem);
  const int S = A.n_swarms;
  // LDS after the tables: per-wave staging lists, per-swarm acceleration [S]
  // (double), region base and capacity [S] (the refills and the finishers
  // read them from here, not from global memory), prefix [S+1], scan scratch
  // [BS], |acceleration| [S] and population-control exponent [S].
  WaveStage* L = reinterpret_cast<WaveStage*>(smem + pic_stage_offset_floats(A.T)) + (threadIdx.x >> 6);
  double* az_d = reinterpret_cast<double*>(reinterpret_cast<WaveStage*>(smem + pic_stage_offset_floats(A.T)) +
                                           BS / 64);
  uint64_t* base_l = reinterpret_cast<uint64_t*>(az_d + S);
  uint64_t* cap_l = base_l + S;
  uint32_t* prefix = (uint32_t*)(cap_l + S);
  uint32_t* tmp = prefix + (S + 1);
  float* az_l = (float*)(tmp + BS);
  int* pck = (int*)(az_l + S);
  __shared__ long long red[kNMom][BS / 64];
  __shared__ unsigned long long acc_lo[kNMom];
  __shared__ long long acc_hi[kNMom];
  for (int s = threadIdx.x; s < S; s += BS) {
    az_d[s] = A.az[s];
    az_l[s] = fabsf((float)A.az[s]);
    base_l[s] = A.base[s];
    cap_l[s] = A.cap_s[s];
  }
  __syncthreads();
  const SwarmField F{az_d, az_l, A.key};
  const auto* ka = (const __attribute__((address_space(4))) SwarmArgs*)__builtin_amdgcn_kernarg_segment_ptr();
  const KArg<EventSink> no_events{&ka->ev};
  const KArg<uint32_t> chunk_k{&ka->chunk};
  const unsigned lane = lane_id();
  const uint32_t wpb = BS / 64;
  SwarmCtl* ctl = A.ctl;

  for (int st = 0; st < A.n_steps; ++st) {
    if (ld_acq(&ctl->stop)) break;
    const int sel = __builtin_amdgcn_readfirstlane(ld_acq(&ctl->cur_sel));  // grid-uniform
    const Soa nxt = A.buf[sel ^ 1];
    const KArg<Soa> cur_k{&ka->buf[sel]}, nxt_k{&ka->buf[sel ^ 1]};
    const uint32_t step = (uint32_t)st;
    for (int s = threadIdx.x; s < S; s += BS) pck[s] = ld_acq(&A.pc_k[s]);
    tile_prefix(A.n_cur, S, 1, prefix, tmp);
    Cnt cnt;
#pragma unroll
    for (int k = 0; k < NCNT; ++k) cnt.v[k] = 0;
    uint32_t psteps = 0;
    const SwarmPlace fin{nxt_k, base_l, cap_l, A.n_nxt, A.cum_att, &ctl->overflow};

    // Phase 1: each swarm's electrons, after population control, from t = 0.
    {
      const BirthSink sink{{&ka->pend[0]}, &ctl->pend[0], A.pend_cap, &ctl->overflow, 0u, no_events};
      const SwarmLoad src{cur_k, base_l, prefix, pck, S, A.key, step, sink, &psteps};
      fly_all<REFILL, ROW, false>((uint64_t)prefix[S], &ctl->take[0], chunk_k, (double)A.dt, F, T, A.S, step, cnt, sink,
                      A.cum_ion, L, src, fin);
    }
    grid.sync();

    // Phase 2: newborns and duplicates of all swarms, generation by generation.
    for (int g = 0;; ++g) {
      const uint64_t np_raw = ld_acq(&ctl->pend[g]);
      if (np_raw == 0) break;
      if (g >= kMaxGenerations) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&ctl->overflow, OVF_LIMIT);
        break;
      }
      const uint64_t np = np_raw < A.pend_cap ? np_raw : A.pend_cap;
      const BirthSink sink{{&ka->pend[(g + 1) & 1]}, &ctl->pend[g + 1], A.pend_cap, &ctl->overflow, 0u, no_events};
      const SwarmPend src{{&ka->pend[g & 1]}};
      fly_all<REFILL, ROW, false>(np, &ctl->take[g + 1], chunk_k, (double)A.dt, F, T, A.S, step, cnt, sink, A.cum_ion, L, src,
                      fin);
      grid.sync();
    }

    // Phase 3: moments of the new population (sample steps), exact sums.
    const bool sample = ((st + 1) % A.sample_every) == 0 && (st + 1) / A.sample_every <= A.n_samples;
    if (sample) {
      const int j = (st + 1) / A.sample_every - 1;
      tile_prefix(A.n_nxt, S, BS, prefix, tmp);
      const uint32_t nt = prefix[S];
      const uint32_t t0 = (uint32_t)(((uint64_t)nt * blockIdx.x) / gridDim.x);
      const uint32_t t1 = (uint32_t)(((uint64_t)nt * (blockIdx.x + 1)) / gridDim.x);
      int cur_s = -1;
      if (threadIdx.x < kNMom) {
        acc_lo[threadIdx.x] = 0;
        acc_hi[threadIdx.x] = 0;
      }
      __syncthreads();
      for (uint32_t tt = t0; tt < t1; ++tt) {
        const int s = find_swarm(prefix, S, tt);
        if (s != cur_s) {
          if (cur_s >= 0 && threadIdx.x < kNMom) {
            unsigned long long* dst = A.mom + (((size_t)cur_s * A.n_samples + j) * kNMom + threadIdx.x) * 2;
            add128_atomic(dst, acc_lo[threadIdx.x], acc_hi[threadIdx.x]);
            acc_lo[threadIdx.x] = 0;
            acc_hi[threadIdx.x] = 0;
          }
          cur_s = s;
          __syncthreads();
        }
        const uint64_t n_s = ld_acq(&A.n_nxt[s]);
        const uint64_t i = (uint64_t)(tt - prefix[s]) * BS + threadIdx.x;
        long long c[kNMom];
#pragma unroll
        for (int m = 0; m < kNMom; ++m) c[m] = 0;
        if (i < n_s) {
          const uint64_t q = base_l[s] + i;
          const double x = nxt.x[q], y = nxt.y[q], z = nxt.z[q];
          const double vx = nxt.vx[q], vy = nxt.vy[q], vz = nxt.vz[q];
          const double v2 = vx * vx + vy * vy + vz * vz;
          const double eps = A.S.k_eps_d * v2;
          double nu_ion = 0.0, nu_att = 0.0;
          {
            float u = fmaf(__log2f((float)eps), T.u_scale, T.u_offset);
            u = fminf(fmaxf(u, 0.0f), (float)(T.n - 1));
            const float fl = fminf(floorf(u), (float)(T.n - 2));
            const int ii = (int)fl;
            const float f = u - fl;
            for (int k = 0; k < T.nproc; ++k) {
              if (eps < (double)T.thr[k]) continue;
              const float nk = lerp_at(A.T.nu + k * T.n, ii, f);
              if (T.kind[k] == IONIZATION) nu_ion += nk;
              if (T.kind[k] == ATTACHMENT) nu_att += nk;
            }
          }
          const double val[kNMom] = {1.0, x, y, z, x * x + y * y, z * z, vx, vy, vz, x * vx + y * vy, z * vz,
                                     eps, nu_ion, nu_att};
#pragma unroll
          for (int m = 0; m < kNMom; ++m) {
            const double v = val[m];
            if (!(fabs(v) < kMomLim[m])) atomicOr(&ctl->overflow, OVF_LIMIT);
            c[m] = __double2ll_rn(ldexp(v, kMomExp[m]));
          }
        }
#pragma unroll
        for (int m = 0; m < kNMom; ++m) {
          long long v = c[m];
          for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
          if (lane == 0) red[m][threadIdx.x >> 6] = v;
        }
        __syncthreads();
        if (threadIdx.x < kNMom) {
          long long b = 0;
          for (uint32_t w = 0; w < wpb; ++w) b += red[threadIdx.x][w];
          unsigned long long lo = acc_lo[threadIdx.x];
          long long hi = acc_hi[threadIdx.x];
          add128(lo, hi, b);
          acc_lo[threadIdx.x] = lo;
          acc_hi[threadIdx.x] = hi;
        }
        __syncthreads();
      }
      if (cur_s >= 0 && threadIdx.x < kNMom) {
        unsigned long long* dst = A.mom + (((size_t)cur_s * A.n_samples + j) * kNMom + threadIdx.x) * 2;
        add128_atomic(dst, acc_lo[threadIdx.x], acc_hi[threadIdx.x]);
      }
    }
    block_counters(cnt, A.partial);
    if (threadIdx.x == 0) A.partial_ps[blockIdx.x] = 0;
    __syncthreads();
    {
      const uint32_t w = wave_sum_u32(psteps);
      if (lane == 0) atomicAdd(&A.partial_ps[blockIdx.x], (unsigned long long)w);
    }
    grid.sync();

    // Commit (block 0): per-swarm counts, sample counters, population control.
    if (blockIdx.x == 0) {
      const unsigned of = ld_acq(&ctl->overflow);
      for (int s = threadIdx.x; s < S; s += BS) {
        const unsigned long long n_new = ld_acq(&A.n_nxt[s]);
        if (sample) {
          const int j = (st + 1) / A.sample_every - 1;
          long long* cc = A.cnt_out + ((size_t)s * A.n_samples + j) * 4;
          cc[0] = (long long)n_new;
          cc[1] = A.L[s];
          cc[2] = (long long)ld_acq(&A.cum_ion[s]);
          cc[3] = (long long)ld_acq(&A.cum_att[s]);
        }
        int k = 0;
        const long long n0 = A.n0[s];
        if (A.pop_control) {
          if ((long long)n_new > 2 * n0) {
            k = 1;
            while (ldexp((double)n_new, -k) > 2.0 * (double)n0) ++k;
            A.L[s] += k;
          } else if (n_new > 0 && 2 * (long long)n_new < n0) {
            k = -1;
            A.L[s] -= 1;
          }
        }
        if (!of) {
          A.pc_k[s] = k;
          A.n_cur[s] = n_new;
        }
        A.n_nxt[s] = 0;
      }
      __shared__ unsigned long long sums[NCNT + 1];
      if (threadIdx.x <= NCNT) sums[threadIdx.x] = 0;
      __syncthreads();
      for (int k = 0; k <= NCNT; ++k) {
        unsigned long long acc = 0;
        for (unsigned b = threadIdx.x; b < gridDim.x; b += BS)
          acc += k < NCNT ? A.partial[(size_t)b * NCNT + k] : A.partial_ps[b];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) atomicAdd(&sums[k], acc);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        if (of) {
          ctl->stop = 1;
          ctl->status = (of & OVF_LIMIT) ? PCMCC_ELIMIT : PCMCC_ECAPACITY;
        } else {
          ctl->cur_sel = sel ^ 1;
          ctl->steps_done += 1;
          ctl->particle_steps += sums[NCNT];
          for (int k = 0; k < NCNT; ++k) ctl->tot[k] += sums[k];
        }
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

// Initial swarms: n0[s] electrons at rest at the origin, ids 0..n0-1.
__global__ void k_swarm_init(Soa buf, const uint64_t* base, const int32_t* n0, int S) {
  for (int s = blockIdx.x; s < S; s += gridDim.x)
    for (int i = threadIdx.x; i < n0[s]; i += blockDim.x) {
      PState p;
      p.x = p.y = p.z = 0.0f;
      p.vx = p.vy = p.vz = 0.0f;
      p.w = 1.0f;
      p.id = (uint64_t)i;
      store_p(buf, base[s] + i, p);
    }
}

// ---------------------------------------------------------------------------
// Estimators (one thread per swarm, double precision).  Window = samples with
// t >= window_start; values over the whole window, errors from batch means
// over n_batches contiguous sub-windows (the first len % B one sample
// longer).  Drift and fluxes are reported along -E (E along +z).
__device__ double mean_of(const double* y, int a0, int a1) {
  double m = 0;
  for (int j = a0; j < a1; ++j) m += y[j];
  return m / (a1 - a0);
}

__device__ double slope_of(const double* t, const double* y, int a0, int a1) {
  const double tm = mean_of(t, a0, a1), ym = mean_of(y, a0, a1);
  double sxy = 0, sxx = 0;
  for (int j = a0; j < a1; ++j) {
    sxy += (t[j] - tm) * (y[j] - ym);
    sxx += (t[j] - tm) * (t[j] - tm);
  }
  return sxy / sxx;
}

__device__ void estimate_range(const double* const* f, int a0, int a1, double E, double* v) {
  const double *tt = f[0], *vz = f[1], *mz = f[2], *cL = f[3], *vzz = f[4], *cT = f[5], *vT = f[6];
  const double *ni = f[7], *na = f[8], *lg = f[9], *ee = f[10];
  v[Q_W_FLUX] = -mean_of(vz, a0, a1);
  v[Q_W_BULK] = -slope_of(tt, mz, a0, a1);
  v[Q_DL_FLUX] = mean_of(cL, a0, a1);
  v[Q_DL_BULK] = 0.5 * slope_of(tt, vzz, a0, a1);
  v[Q_DT_FLUX] = 0.5 * mean_of(cT, a0, a1);
  v[Q_DT_BULK] = 0.25 * slope_of(tt, vT, a0, a1);
  v[Q_NU_ION] = mean_of(ni, a0, a1);
  v[Q_NU_ATT] = mean_of(na, a0, a1);
  v[Q_NU_EFF] = slope_of(tt, lg, a0, a1);
  v[Q_MEAN_EPS] = mean_of(ee, a0, a1);
  v[Q_MU] = v[Q_W_FLUX] / E;
  v[Q_ALPHA] = v[Q_NU_ION] / v[Q_W_FLUX];
  v[Q_ETA] = v[Q_NU_ATT] / v[Q_W_FLUX];
  v[Q_RATIO] = v[Q_W_BULK] / v[Q_W_FLUX];
}

__global__ void k_swarm_estimate(const unsigned long long* mom, const long long* cnt, int S, int J, double dt_sample,
                                 double t_window, int n_batches, const double* EN, double gas_N, double* values,
                                 double* errors, double* work) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S) return;
  double* w = work + (size_t)s * 11 * J;
  const double* f[11];
  for (int k = 0; k < 11; ++k) f[k] = w + (size_t)k * J;
  double *tt = w, *vz = w + J, *mz = w + 2 * J, *cL = w + 3 * J, *vzz = w + 4 * J, *cT = w + 5 * J, *vT = w + 6 * J;
  double *ni = w + 7 * J, *na = w + 8 * J, *lg = w + 9 * J, *ee = w + 10 * J;
  bool empty = false;
  int j0 = J;
  for (int j = 0; j < J; ++j) {
    tt[j] = (j + 1) * dt_sample;
    if (j0 == J && tt[j] >= t_window * (1.0 - 1e-12)) j0 = j;
    double m[kNMom];
    for (int k = 0; k < kNMom; ++k) {
      const unsigned long long lo = mom[(((size_t)s * J + j) * kNMom + k) * 2];
      const long long hi = (long long)mom[(((size_t)s * J + j) * kNMom + k) * 2 + 1];
      m[k] = ldexp((double)hi * 18446744073709551616.0 + (double)lo, -kMomExp[k]);
    }
    const double n = m[0];
    const long long* c = cnt + ((size_t)s * J + j) * 4;
    if (!(n > 0)) {
      if (j >= j0) empty = true;
      continue;
    }
    const double mx = m[1] / n, my = m[2] / n, zz = m[3] / n;
    const double vxm = m[6] / n, vym = m[7] / n, vzm = m[8] / n;
    vz[j] = vzm;
    mz[j] = zz;
    cL[j] = m[10] / n - zz * vzm;
    vzz[j] = m[5] / n - zz * zz;
    cT[j] = m[9] / n - mx * vxm - my * vym;
    vT[j] = m[4] / n - mx * mx - my * my;
    ni[j] = m[12] / n;
    na[j] = m[13] / n;
    lg[j] = log(n) + (double)c[1] * 0.69314718055994530942;
    ee[j] = m[11] / n;
  }
  const double E = EN[s] * 1e-21 * gas_N;
  const int len = J - j0;
  double v[kNQ];
  if (empty || len < 2 * n_batches || n_batches < 2) {
    for (int k = 0; k < kNQ; ++k) {
      values[(size_t)s * kNQ + k] = NAN;
      errors[(size_t)s * kNQ + k] = NAN;
    }
    return;
  }
  estimate_range(f, j0, J, E, v);
  for (int k = 0; k < kNQ; ++k) values[(size_t)s * kNQ + k] = v[k];
  double s1[kNQ], s2[kNQ];
  for (int k = 0; k < kNQ; ++k) s1[k] = s2[k] = 0.0;
  const int q = len / n_batches, r = len % n_batches;
  for (int b = 0; b < n_batches; ++b) {
    const int a0 = j0 + b * q + min(b, r);
    const int a1 = a0 + q + (b < r ? 1 : 0);
    estimate_range(f, a0, a1, E, v);
    for (int k = 0; k < kNQ; ++k) {
      s1[k] += v[k];
      s2[k] += v[k] * v[k];
    }
  }
  for (int k = 0; k < kNQ; ++k) {
    const double B = n_batches;
    const double var = (s2[k] - s1[k] * s1[k] / B) / (B - 1.0);
    errors[(size_t)s * kNQ + k] = sqrt(fmax(var, 0.0) / B);
  }
}

// ---------------------------------------------------------------------------
size_t swarm_lds_bytes(const TableView& T, int S, int block) {
  return pic_stage_offset_floats(T) * sizeof(float) + (size_t)(block / 64) * sizeof(WaveStage) + (size_t)S * 8 +
         (size_t)S * 16 + (size_t)(S + 1) * 4 + (size_t)block * 4 + (size_t)S * 4 + (size_t)S * 4;
}

template <int BS, int ROW>
static const void* swarm_kernel_r(int refill) {
  switch (refill) {
    case 16: return (const void*)k_swarm_steps<BS, 16, ROW>;
    case 24: return (const void*)k_swarm_steps<BS, 24, ROW>;
    case 32: return (const void*)k_swarm_steps<BS, 32, ROW>;
    default: return nullptr;
  }
}

template <int ROW>
static const void* swarm_kernel_b(int block, int refill) {
  switch (block) {
    case 64: return swarm_kernel_r<64, ROW>(refill);
    case 128: return swarm_kernel_r<128, ROW>(refill);
    case 256: return swarm_kernel_r<256, ROW>(refill);
    case 512: return swarm_kernel_r<512, ROW>(refill);
    default: return nullptr;
  }
}

static const void* swarm_kernel(int block, int refill, int row) {
  return row == 4 ? swarm_kernel_b<4>(block, refill) : row == 8 ? swarm_kernel_b<8>(block, refill) : nullptr;
}

hipError_t occupancy_swarm_steps(int block, int refill, int row, size_t lds, int* blocks_per_cu) {
  const void* k = swarm_kernel(block, refill, row);
  if (!k) return hipErrorInvalidValue;
  return coresident_blocks(k, block, lds, blocks_per_cu);
}

hipError_t launch_swarm_steps(const SwarmArgs& args, int grid, int block, int refill, hipStream_t stream) {
  const void* k = swarm_kernel(block, refill, table_row(args.T.nproc));
  if (!k) return hipErrorInvalidValue;
  void* kargs[] = {(void*)&args};
  return hipLaunchCooperativeKernel(k, dim3(grid), dim3(block), kargs,
                                    (unsigned)swarm_lds_bytes(args.T, args.n_swarms, block), stream);
}

hipError_t launch_swarm_init(const Soa& buf, const uint64_t* base, const int32_t* n0, int S, hipStream_t stream) {
  hipLaunchKernelGGL(k_swarm_init, dim3(std::min(S, 4096)), dim3(256), 0, stream, buf, base, n0, S);
  return hipGetLastError();
}

hipError_t launch_swarm_estimate(const unsigned long long* mom, const long long* cnt, int S, int J, double dt_sample,
                                 double t_window, int n_batches, const double* EN, double gas_N, double* values,
                                 double* errors, double* work, hipStream_t stream) {
  hipLaunchKernelGGL(k_swarm_estimate, dim3((S + 63) / 64), dim3(64), 0, stream, mom, cnt, S, J, dt_sample, t_window,
                     n_batches, EN, gas_N, values, errors, work);
  return hipGetLastError();
}

}  // namespace pcmcc
