// Segment-pipelined electron mover of the PIC step and the swarms.
//
// Method: arXiv:2110.14494 Sec. 2.1.1 (velocity Verlet, eq. (1)-(2), and the
// null-collision method) and Sec. 2.1.5 (tabulated rates).  Per electron
// and step: from its start time, flight segments of length min(tau, horizon,
// rest of the step), tau = -ln(U)/nu_hat with nu_hat the majorant of the total
// rate for the speeds reachable within the horizon; at the end of a segment
// that did not reach the horizon, the process is chosen from the cumulative
// rates at the electron's energy (null if none or below its threshold) and
// applied: isotropic scattering with the elastic recoil loss, excitation
// losing its threshold, ionization sharing the remaining energy equally with
// a newborn, attachment removing the electron.  Random numbers are
// Philox4x32-10 keyed by the run (and group) with counter (id, step, segment,
// purpose), so results do not depend on the schedule.
//
// Schedule: a lane holds one electron.  Every iteration of a wave's loop does
// exactly one field gather per lane (at the end point of the lane's pending
// flight segment, or at the start point of a freshly loaded electron), then
// completes that segment (second half of the Verlet update, then the
// collision if the segment ended in one), plans the next segment (majorant,
// free-flight time) and moves the position to its end.  An electron that
// reaches the end of the step, is attached or hits the segment limit parks
// in its lane; once REFILL lanes are free, the parked electrons are
// written out and the free lanes take new electrons from a grid-wide work
// counter, all in one batch.  Lanes therefore stay busy regardless of how
// many segments each electron needs within the step, the gather (the only
// global-memory read of a segment) is one instruction stream for the whole
// wave, and the rare per-electron work (start, finish, building a newborn)
// runs in batches instead of with one or two lanes active.
#pragma once

#include "pcmcc_internal.hpp"
#include "pcmcc_mover.hpp"

namespace pcmcc {

enum FlightMode : int { FM_IDLE = 0, FM_NEW = 1, FM_FLY = 2, FM_DONE = 3 };
enum Segment : int { SEG_END = 0, SEG_HORIZON = 1, SEG_COLLIDE = 2 };
enum FlightEvent : int { EV_GO = 0, EV_DONE = 1, EV_ATTACHED = 2, EV_LIMIT = 3 };

// Schedule of the mover (kRefillChoices, kChunkMin, kChunkMax): REFILL, a
// template parameter of fly_all, is the number of free lanes that triggers
// a finish-and-refill batch (few: the batch runs often with few lanes;
// many: lanes idle longer before it); the chunk is the number of electrons
// a wave takes from the work counter at a time (small: more atomics; large:
// a longer tail at the end of a phase).

// Per-wave staging lists in LDS.  Newborns, holes and placed newborns are
// collected per wave and written out kFlushAt or more at a time, each batch
// with one global atomic: events are frequent (about one newborn per
// hundred flight segments in a streamer head), and a device-wide atomic per
// event and wave saturates the memory-side atomic unit.  An event that finds
// its list full (more than kStage - kFlushAt events of one wave in one
// iteration) takes the direct path with its own atomic.
constexpr uint32_t kStage = 64;
constexpr uint32_t kFlushAt = 48;  // (tuned: 32 -> 670 ms, 48 -> 657 ms per streamer call)

struct WaveStage {
  // newborns as their parent left them: x, y, z, w, birth time; segment
  // number, group, parent id and the newborn's energy (the rest is drawn at
  // flush)
  float b[5][kStage];
  uint32_t bj[kStage];
  uint32_t btag[kStage];
  uint64_t bpid[kStage];
  double beps[kStage];
  // finished electrons: x .. w, group, id (phase 1 of the PIC step: s[0]
  // holds hole slots)
  float s[7][kStage];
  uint32_t stag[kStage];
  uint64_t sid[kStage];
};

// Whole wave: for the lanes with `active` set, reserves one slot each in the
// counter ctr[tag] of the lane's group, with one atomic per distinct group
// present; returns the lane's slot (undefined for inactive lanes).  The
// groups are found first (ballots only); then every group's leader (its
// lowest lane) issues its atomic in the same instruction, so the wave waits
// for one round trip however many groups it holds, and each lane takes its
// leader's base by a lane shuffle.
__device__ __forceinline__ uint64_t group_reserve(unsigned long long* ctr, uint32_t tag, bool active) {
  uint64_t pending = __ballot(active);
  const uint32_t lane = lane_id();
  int leader_of = 0;
  uint32_t rank = 0, count = 0;
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t t = __builtin_amdgcn_readlane(tag, leader);
    const uint64_t m = __ballot(active && tag == t) & pending;
    if ((m >> lane) & 1) {
      leader_of = leader;
      rank = rank_in(m);
    }
    if ((int)lane == leader) count = (uint32_t)__popcll(m);
    pending &= ~m;
  }
  unsigned long long base = 0;
  if (active && rank == 0) base = atomicAdd(&ctr[tag], (unsigned long long)count);
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)base, leader_of);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(base >> 32), leader_of);
  return (((uint64_t)hi << 32) | lo) + rank;
}

// Whole wave: adds, per distinct group among the lanes with `active` set, the
// number of such lanes to ctr[tag] (one atomic per group).
__device__ __forceinline__ void group_count(unsigned long long* ctr, uint32_t tag, bool active) {
  uint64_t pending = __ballot(active);
  const uint32_t lane = lane_id();
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t t = __builtin_amdgcn_readlane(tag, leader);
    const uint64_t m = __ballot(active && tag == t) & pending;
    if ((int)lane == leader) atomicAdd(&ctr[t], (unsigned long long)__popcll(m));
    pending &= ~m;
  }
}

// Offset (in floats) of the staging lists after the staged tables in the
// step kernel's LDS, 16-byte aligned.
__host__ __device__ inline size_t pic_stage_offset_floats(const TableView& T) {
  return (table_lds_floats(T) + 3) & ~(size_t)3;
}

// Id and velocity of the newborn of an ionization: the birth draw of the
// parent's segment gives the id (first two words) and an isotropic
// direction, the speed follows from the newborn's energy.
__device__ __forceinline__ void make_child(Key key, uint32_t step, const SpeciesView& S, uint64_t pid, uint32_t j,
                                           double eps_new, PState& c) {
  const uint4 b = draw(key, pid, step, j, TAG_BIRTH);
  c.id = (uint64_t)b.x | ((uint64_t)b.y << 32);
  double cx, cy, cz;
  iso_dir(b.z, b.w, cx, cy, cz);
  const double cs = sqrt_nr(eps_new * S.inv_k_d);
  c.vx = (float)(cs * cx);
  c.vy = (float)(cs * cy);
  c.vz = (float)(cs * cz);
}

// Newborn queue of a phase seen through the wave's staging list.  Field
// supplies the random-number key of an electron's group; the queue records
// the group of each newborn when it has a group array, and cum_ion (if not
// null) counts ionizations per group.
template <class Field>
struct StagedBirths {
  WaveStage* L;
  BirthSink q;  // global queue: flushes and direct pushes
  const Field& F;
  uint32_t step;
  SpeciesView S;
  unsigned long long* cum_ion;
  uint32_t n;  // staged entries (wave-uniform)

  // Called by the lanes that create a newborn; returns true if it was staged.
  __device__ __forceinline__ bool push(float x, float y, float z, float w, float tb, uint32_t tag, uint64_t pid,
                                       uint32_t j, double eps_new) const {
    const uint32_t s = n + rank_in(__ballot(1));
    if (s < kStage) {
      L->b[0][s] = x;
      L->b[1][s] = y;
      L->b[2][s] = z;
      L->b[3][s] = w;
      L->b[4][s] = tb;
      L->bj[s] = j;
      L->btag[s] = tag;
      L->bpid[s] = pid;
      L->beps[s] = eps_new;
      return true;
    }
    PState c;
    c.x = x;
    c.y = y;
    c.z = z;
    c.w = w;
    make_child(F.key(tag), step, S, pid, j, eps_new, c);
    BirthSink qt = q;
    qt.tag = tag;
    qt.push(c, tb);
    if (cum_ion) atomicAdd(&cum_ion[tag], 1ull);
    const EventSink ev = q.evk.get();
    if (ev.ix) {
      const uint64_t es = wave_reserve(ev.n);
      if (es < ev.cap) {
        ev.ix[es] = x;
        ev.iy[es] = y;
        ev.iz[es] = z;
        ev.iw[es] = w;
      } else {
        atomicOr(ev.overflow, OVF_CAPACITY);
      }
    }
    return false;
  }

  // Whole wave: builds the staged newborns and writes them to the queue.
  __device__ __forceinline__ void flush() {
    if (n == 0) return;
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(q.count, (unsigned long long)n);
    const uint64_t b = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32)) << 32) |
                       __builtin_amdgcn_readfirstlane((uint32_t)base);
    const uint32_t l = lane_id();
    const bool mine = l < n;
    const uint32_t tag = mine ? L->btag[l] : 0u;
    if (mine) {
      const uint64_t slot = b + l;
      if (slot < q.cap) {
        PState c;
        make_child(F.key(tag), step, S, L->bpid[l], L->bj[l], L->beps[l], c);
        const PendSoa Q = q.qk.get();
        if (Q.sw) Q.sw[slot] = tag;
        Q.x[slot] = L->b[0][l];
        Q.y[slot] = L->b[1][l];
        Q.z[slot] = L->b[2][l];
        Q.vx[slot] = c.vx;
        Q.vy[slot] = c.vy;
        Q.vz[slot] = c.vz;
        Q.w[slot] = L->b[3][l];
        Q.tb[slot] = L->b[4][l];
        Q.id[slot] = c.id;
      } else {
        atomicOr(q.overflow, OVF_CAPACITY);
      }
    }
    if (cum_ion) group_count(cum_ion, tag, mine);
    const EventSink ev = q.evk.get();
    if (ev.ix) {  // the positive ions of the flushed births
      unsigned long long eb = 0;
      if (lane_id() == 0) eb = atomicAdd(ev.n, (unsigned long long)n);
      const uint64_t e0 = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(eb >> 32)) << 32) |
                          __builtin_amdgcn_readfirstlane((uint32_t)eb);
      if (mine) {
        const uint64_t es = e0 + l;
        if (es < ev.cap) {
          ev.ix[es] = L->b[0][l];
          ev.iy[es] = L->b[1][l];
          ev.iz[es] = L->b[2][l];
          ev.iw[es] = L->b[3][l];
        } else {
          atomicOr(ev.overflow, OVF_CAPACITY);
        }
      }
    }
    n = 0;
  }
};

struct Flight {
  double x, y, z, vx, vy, vz, ax, ay, az;
  double t;  // time within the step
  double h;  // length of the pending segment
  float a_abs, da, w, nu_hat;
  uint64_t id;
  uint32_t j;           // number of the next segment (random-number counter)
  uint32_t src;         // slot the electron came from
  uint32_t r1, r2, r3;  // uniforms of the pending collision
  uint32_t tag;         // group of the electron (swarm index; 0 in the PIC step)
  PhiloxPre pre;        // the products its draws of this step share
  int mode;
  int seg;  // kind of the pending segment; for a parked electron, its event
};

__device__ __forceinline__ PState flight_record(const Flight& f) {
  PState p;
  p.x = (float)f.x;
  p.y = (float)f.y;
  p.z = (float)f.z;
  p.vx = (float)f.vx;
  p.vy = (float)f.vy;
  p.vz = (float)f.vz;
  p.w = f.w;
  p.id = f.id;
  p.xd = f.x;
  p.yd = f.y;
  p.zd = f.z;
  return p;
}

__device__ __forceinline__ void flight_start(Flight& f, const PState& p, double t0, uint32_t src,
                                             uint32_t tag = 0) {
  f.x = p.x;
  f.y = p.y;
  f.z = p.z;
  f.vx = p.vx;
  f.vy = p.vy;
  f.vz = p.vz;
  f.w = p.w;
  f.id = p.id;
  f.t = t0;
  f.src = src;
  f.tag = tag;
  f.j = 0;
  f.mode = FM_NEW;
}

// Draws the next segment from the current state (acceleration valid at the
// current position): majorant, horizon, free-flight time; then moves the
// position to the segment's end (first half of the Verlet update).
__device__ __forceinline__ int flight_plan(Flight& f, double dt, const Tab& T, const SpeciesView& S, Key key,
                                           uint32_t step, Cnt& cnt) {
  if (f.j >= (uint32_t)kMaxSegments) {
    cnt.v[C_ERR]++;
    return EV_LIMIT;
  }
  const uint4 r = draw_pre(key, f.pre, step, (f.j << 2) | TAG_MAIN);
  f.j++;
  cnt.v[C_TRIALS]++;
  const double t_rem = dt - f.t;
  const float3 vf = make_float3((float)f.vx, (float)f.vy, (float)f.vz);
  const float3 af = make_float3((float)f.ax, (float)f.ay, (float)f.az);
  // Single-precision square roots and reciprocals to about one ulp: the
  // majorant's 2^-16 guard covers them, and the free-flight time only needs
  // single precision.
  const float speed = __builtin_amdgcn_sqrtf(fmaf(vf.z, vf.z, fmaf(vf.y, vf.y, vf.x * vf.x)));
  const TabConst tc = tab_const();
  const float nu_full = majorant_t(T, tc, speed_bound(vf, af, speed, f.a_abs, f.da, (float)t_rem));
  const bool limited = kKappa < nu_full * (float)t_rem;
  // Where any lane of the wave is limited, both majorants are evaluated and
  // one is selected, which keeps the lanes on one path (nu_full = 0 gives an
  // unused, finite lookup); a wave without a limited lane skips the second.
  float h_lim = 0.0f, nu_lim = 0.0f;
  if (__ballot(limited) != 0) {
    h_lim = kKappa * __builtin_amdgcn_rcpf(nu_full);
    nu_lim = majorant_t(T, tc, speed_bound(vf, af, speed, f.a_abs, f.da, h_lim));
  }
  const double h = limited ? (double)h_lim : t_rem;
  const float nu_hat = limited ? nu_lim : nu_full;
  // ln U from the hardware base-2 logarithm (U in [2^-24, 1) is never
  // subnormal; within 1.2e-7 relative of ln U over all 2^23 uniforms)
  const float ln_u = __builtin_amdgcn_logf(unif(r.x)) * 0.693147182f;
  const double tau = nu_hat > 0.0f ? (double)(-ln_u * __builtin_amdgcn_rcpf(nu_hat)) : (double)INFINITY;
  double hs;
  if (tau >= h) {
    hs = h;
    f.seg = limited ? SEG_HORIZON : SEG_END;
  } else {
    hs = tau;
    f.seg = SEG_COLLIDE;
  }
  f.r1 = r.y;
  f.r2 = r.z;
  f.r3 = r.w;
  f.nu_hat = nu_hat;
  f.h = hs;
  f.x = fma(hs, fma(0.5 * f.ax, hs, f.vx), f.x);
  f.y = fma(hs, fma(0.5 * f.ay, hs, f.vy), f.y);
  f.z = fma(hs, fma(0.5 * f.az, hs, f.vz), f.z);
  if (f.seg != SEG_END) f.t += hs;
  return EV_GO;
}

// Completes the pending segment with the acceleration `an` gathered at its
// end point, then applies its collision, if any.
template <int ROW, class Field>
__device__ __forceinline__ int flight_complete(Flight& f, const double3 an, const Tab& T, const SpeciesView& S,
                                               Cnt& cnt, const StagedBirths<Field>& births, bool& staged) {
  const double hh = 0.5 * f.h;
  f.vx = fma(f.ax + an.x, hh, f.vx);
  f.vy = fma(f.ay + an.y, hh, f.vy);
  f.vz = fma(f.az + an.z, hh, f.vz);
  f.ax = an.x;
  f.ay = an.y;
  f.az = an.z;
  // The outcome is formed with selects over the whole wave: the candidate
  // lookup, the direction and the new energy are evaluated on every lane (a
  // wave almost always holds lanes of each kind, so masking would save no
  // issue slots) and applied where they hold; only the staged newborn is a
  // branch.  A lane takes exactly the values the branchy form would give it.
  const bool cand = f.seg == SEG_COLLIDE;
  int ev = f.seg == SEG_END ? EV_DONE : EV_GO;
  // a wave without a candidate (sparse waves: small populations, the ends
  // of phases) skips the collision work
  if (__ballot(cand) == 0) return ev;

  // Candidate collision: real process k, or null.
  const TabConst tc = tab_const();
  const double v2 = fma(f.vz, f.vz, fma(f.vy, f.vy, f.vx * f.vx));
  const double eps = tc.k_eps_d * v2;
  float u = fmaf(__log2f((float)eps), tc.u_scale, tc.u_offset);
  u = clamp_med3(u, 0.0f, tc.u_top);
  const float fl = clamp_med3(floorf(u), 0.0f, tc.fl_top);
  const int i = (int)fl;
  const float fr = u - fl;
  const float yv = unif(f.r1) * f.nu_hat;
  float cum[ROW];
  cum_rates_row<ROW>(T, i, fr, cum);
  // the total rate (the largest cumulative entry; padding entries are zero)
  // must not exceed the majorant
  float tot = cum[0];
#pragma unroll
  for (int kk = 1; kk < ROW; ++kk) tot = fmaxf(tot, cum[kk]);
  cnt.v[C_MAJ] += cand && tot > f.nu_hat;
  const int k = pick_process_row<ROW>(cum, yv);
  const int ks = k < 0 ? 0 : k;
  const double thr = (double)T.thr[ks];
  const bool real = cand && k >= 0 && !(eps < thr);
  cnt.v[C_NULL] += cand && !real;
  cnt.v[C_OOT] += real && eps > tc.eps_max;
  const int kind = T.kind[ks];
  cnt.v[C_EL] += real && kind == ELASTIC;
  cnt.v[C_EXC] += real && kind == EXCITATION;
  cnt.v[C_ION] += real && kind == IONIZATION;
  cnt.v[C_ATT] += real && kind == ATTACHMENT;
  if (real && kind == ATTACHMENT) ev = EV_ATTACHED;
  const bool scatter = real && kind != ATTACHMENT;

  double nx, ny, nz;
  iso_dir(f.r2, f.r3, nx, ny, nz);
  const double cchi = v2 > 0.0 ? fma(f.vz, nz, fma(f.vy, ny, f.vx * nx)) * rsqrt_nr(v2) : 0.0;
  const double eps_el = eps * fma(-(double)tc.recoil, 1.0 - cchi, 1.0);
  const double eps_ion = 0.5 * (eps - thr);
  const double eps_new = kind == ELASTIC ? eps_el : (kind == EXCITATION ? eps - thr : eps_ion);
  if (scatter && kind == IONIZATION)
    staged = births.push((float)f.x, (float)f.y, (float)f.z, f.w, (float)f.t, f.tag, f.id, f.j - 1, eps_ion);
  const double sn = sqrt_nr(eps_new * tc.inv_k_d);
  f.vx = scatter ? sn * nx : f.vx;
  f.vy = scatter ? sn * ny : f.vy;
  f.vz = scatter ? sn * nz : f.vz;
  return ev;
}

// Runs every electron of a source (n of them) through the rest of the step
// (tables of ROW floats per node, table_row(nproc)),
// REFILL lanes at a time (see above), `chunk` (a power of two in [kChunkMin,
// kChunkMax], read from the kernel arguments) electrons per work-counter
// grab, or with GUIDED a shrinking share of the rest down to kChunkMin.
// Field: key(tag) gives the random-number key of a group, accel(x, y, z,
// tag, where) the acceleration (and where the field was read), bound_at(where,
// tag, speed, t_rem, a_abs, da) the field bounds for the rest of the step.
// Source: load(i, Flight&, hint) starts electron i (or leaves the lane
// idle); hint(first) is computed once per chunk taken (wave-uniform) and
// passed to the loads of its electrons.
// Finish: done_all(Flight&, parked, Cnt&, WaveStage*, staged count) takes the
// electrons that left the step (called by the whole wave; `parked` marks the
// lanes holding one, f.seg is its event) and returns the new staged count
// (it may flush on its own), flush(WaveStage*, count) writes out the wave's
// staged results; can_open() tells whether the wave may take another chunk
// of work, open_chunk(first, size) registers a chunk it took and returns its
// tag, which tag(Flight&, tag) gives each electron loaded from it.  Must be called by whole waves with wave-uniform
// arguments; `take` is the grid-wide work counter (zero before the first
// wave starts).  cum_ion (nullable) counts ionizations per group.  Every
// staged entry is written out before the function returns.
template <int REFILL, int ROW, bool GUIDED, class Field, class Source, class Finish>
__device__ __forceinline__ void fly_all(uint64_t n, unsigned long long* take, KArg<uint32_t> chunk, double dt,
                                        const Field& F, const Tab& T, const SpeciesView& S, uint32_t step, Cnt& cnt,
                                        const BirthSink& sink, unsigned long long* cum_ion, WaveStage* L,
                                        const Source& source, const Finish& finish) {
  Flight f;
  f.mode = FM_IDLE;
  StagedBirths<Field> births{L, sink, F, step, S, cum_ion, 0u};
  uint32_t n_done = 0;  // entries of the finish list
  uint64_t pool_next = 0, pool_end = 0;
  uint64_t seen = 0;  // the work counter after this wave's previous grab
  uint32_t chunk_tag = 0;  // finisher's tag of the current chunk
  uint32_t src_hint = 0;   // source's hint for the current chunk
  bool dry = n == 0;
  const uint32_t lane = lane_id();
  for (;;) {
    const uint64_t busy = __ballot(f.mode == FM_FLY);
    if (64u - (uint32_t)__popcll(busy) >= (uint32_t)REFILL || busy == 0) {
      // Finish the parked electrons (room for all of them in the list).
      const uint32_t n_fin = (uint32_t)__popcll(__ballot(f.mode == FM_DONE));
      if (n_fin > 0) {
        if (n_done + n_fin > kStage) {
          finish.flush(L, n_done);
          n_done = 0;
        }
        n_done = finish.done_all(f, f.mode == FM_DONE, cnt, L, n_done);
        if (f.mode == FM_DONE) f.mode = FM_IDLE;
        if (n_done >= kFlushAt) {
          finish.flush(L, n_done);
          n_done = 0;
        }
      }
      // Start new electrons in the free lanes.
      if (!dry) {
        const uint64_t idle = __ballot(f.mode == FM_IDLE);
        const uint32_t n_idle = (uint32_t)__popcll(idle);
        const uint32_t rank = rank_in(idle);
        uint32_t served = 0;
        while (served < n_idle) {
          if (pool_next == pool_end) {
            if (!finish.can_open()) break;  // the lanes stay idle until a chunk of this wave completes
            // GUIDED: a share of what was left at this wave's previous grab,
            // (n - seen) / (2 waves), between kChunkMin and the schedule's
            // chunk, so that a phase ends on small chunks instead of leaving
            // one wave a whole large chunk behind the others (the PIC step:
            // 1 % on its large phases; the swarms' short steps lose more to
            // the extra grabs than they gain).
            uint32_t ch = chunk.get();
            if (GUIDED && seen > 0) {
              const uint64_t waves = (uint64_t)gridDim.x * blockDim.x / 64u;
              const uint64_t share = seen < n ? (n - seen) / (2u * waves) : 0u;
              ch = share < (uint64_t)kChunkMin ? (uint32_t)kChunkMin : (share < ch ? (uint32_t)share : ch);
            }
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(take, (unsigned long long)ch);
            const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
            const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
            const uint64_t b = ((uint64_t)hi << 32) | lo;
            seen = b + ch;
            if (b >= n) {
              dry = true;
              break;
            }
            pool_next = b;
            pool_end = b + ch < n ? b + ch : n;
            chunk_tag = finish.open_chunk(b, (uint32_t)(pool_end - b));
            src_hint = source.hint(b);
          }
          const uint32_t avail = (uint32_t)(pool_end - pool_next);
          const uint32_t got = avail < n_idle - served ? avail : n_idle - served;
          if (f.mode == FM_IDLE && rank >= served && rank < served + got) {
            source.load(pool_next + (rank - served), f, src_hint);
            finish.tag(f, chunk_tag);
            if (f.mode == FM_NEW) f.pre = philox_pre(F.key(f.tag), f.id, step);
          }
          pool_next += got;
          served += got;
        }
      }
    }
    // Leave only when the work counter is exhausted: a refill may leave every
    // lane idle (a swarm's population control drops the electrons it loads),
    // and the next iteration then refills again.
    if (dry && __ballot(f.mode != FM_IDLE) == 0) break;
    bool born = false;
    if (f.mode == FM_FLY || f.mode == FM_NEW) {
      typename Field::Where where;
      const double3 an = F.accel(f.x, f.y, f.z, f.tag, where);
      int ev;
      if (f.mode == FM_NEW) {
        // start of the electron's flight: acceleration and field bound for
        // the rest of the step (the bound from the record just gathered)
        f.ax = an.x;
        f.ay = an.y;
        f.az = an.z;
        F.bound_at(where, f.tag, __builtin_amdgcn_sqrtf((float)fma(f.vz, f.vz, fma(f.vy, f.vy, f.vx * f.vx))),
                   (float)(dt - f.t), f.a_abs, f.da);
        f.mode = FM_FLY;
        ev = EV_GO;
      } else {
        ev = flight_complete<ROW>(f, an, T, S, cnt, births, born);
      }
      if (ev == EV_GO) ev = flight_plan(f, dt, T, S, F.key(f.tag), step, cnt);
      if (ev != EV_GO) {
        f.mode = FM_DONE;
        f.seg = ev;
      }
    }
    // Whole wave again: count the staged newborns, write out a full list.
    births.n += (uint32_t)__popcll(__ballot(born));
    if (births.n >= kFlushAt) births.flush();
  }
  births.flush();
  if (n_done > 0) finish.flush(L, n_done);
}

}  // namespace pcmcc
