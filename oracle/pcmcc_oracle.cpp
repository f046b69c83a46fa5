// Plain FP64 CPU oracle for the PIC-MCC electron update and the uniform-field
// swarm.  TEST INFRASTRUCTURE ONLY: it is loaded by the tests, by the smoke
// check and by the CPU-baseline leg of the benchmark, never by the product
// library.  It shares no code, header or table with the HIP path; the two
// meet only in the seeded input arrays and in the published definition of
// Philox4x32-10 that each side implements on its own.
//
// Written for readability, not speed: every quantity in double precision,
// one particle at a time, in the order the method states.  Built with
// -ffp-contract=off so that the deposit (a plain integer sum) is reproducible
// bit for bit.
//
// Paper: Wang, Sun, Teunissen, "A comparison of particle and fluid models for
// positive streamer discharges in air" (arXiv:2110.14494).
//   * mover: velocity Verlet, Sec. 2.1.1 eq. (1)-(2); the velocity update is
//     read as v += (dt/2) [a(t) + a(t+dt)] (the printed form drops dt);
//   * collisions: null-collision method, Sec. 2.1.1, with rates from cross
//     sections, Sec. 2.1.5;
//   * field interpolation and density mapping: trilinear (CIC) on the
//     cell-centred grid, Sec. 2.1.3; homogeneous Neumann density boundaries,
//     Sec. 2.3;
//   * flux and bulk swarm coefficients from uniform-field Monte Carlo,
//     Sec. 2.2.2 (the estimators themselves live in estimators.py).
// Where the paper is silent (scattering law, energy sharing, majorant, random
// number layout) the reading taken is stated next to the code.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

int orc_deposit_impl(const float* x, const float* y, const float* z, const float* w, int64_t n, int nx, int ny,
                     int nz, double x0, double y0, double z0, double inv_dx, int64_t* rho);
// A charge outside the fixed-point range of the deposit.
constexpr int ORC_ERANGE = -8;

namespace {

constexpr double kEV = 1.602176634e-19;  // J per eV (exact SI value)
constexpr double kPI = 3.14159265358979323846;

enum Kind { ELASTIC = 0, EXCITATION = 1, IONIZATION = 2, ATTACHMENT = 3 };
enum Flags { EFFECTIVE_TO_ELASTIC = 1, RATES = 2 };
enum Tag { TAG_MAIN = 0, TAG_BIRTH = 1, TAG_AUX = 2, TAG_WEIGHT = 3 };

// Upper limit on flight segments of one particle within one step; a particle
// reaching it is dropped and counted as an error (guards a runaway loop).
constexpr int kMaxSegments = 1 << 20;

// Flight horizon: a segment's majorant covers at most KAPPA / nu_full of time
// (nu_full = the majorant for the whole rest of the step), about KAPPA
// candidate collisions; a flight that outlasts the horizon ends there and a
// new candidate time is drawn (exact, the exponential law being memoryless).
constexpr double KAPPA = 4.0;

// Test knob: 1 replaces the majorant rule by the plain constant bound (the
// largest total rate in the table, no horizon), for checks that the rule
// leaves the physics unchanged.
int g_constant_majorant = 0;

// Test knob that plants a known mistake in the majorant rule, so that the
// tests can show the violation counter detects a wrong bound: 1 drops the
// field-range term of the speed bound (as if the field did not change along
// the flight), 2 takes nine tenths of every majorant.  0 = the rule as stated.
int g_majorant_fault = 0;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the
// round keys bumped by the Weyl constants between rounds.
void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t p0 = (uint64_t)M0 * c[0];
    const uint64_t p1 = (uint64_t)M1 * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
  }
}

// Draw for (particle id, absolute step, segment j, tag).
struct Draw {
  uint32_t r[4];
};
Draw draw(uint32_t key0, uint32_t key1, uint64_t id, uint64_t step, uint32_t j, uint32_t tag) {
  Draw d;
  d.r[0] = (uint32_t)id;
  d.r[1] = (uint32_t)(id >> 32);
  d.r[2] = (uint32_t)step;
  d.r[3] = (j << 2) | tag;
  philox4x32_10(d.r, key0, key1);
  return d;
}

// Uniform in (0,1) from the top 23 bits; exact in single and double precision.
double unif(uint32_t r) { return ((double)(r >> 9) + 0.5) * 0x1p-23; }

// ---------------------------------------------------------------------------
struct Species {
  double m, q, N, M;
  double k_eps;  // eps[eV] = k_eps * |v|^2
};

struct Tables {
  int n = 0, nproc = 0;
  double lnmin = 0, dlog = 0, eps_max = 0;
  std::vector<int> kind;
  std::vector<double> thr;
  std::vector<double> nu;  // [nproc][n] per-process collision frequency at nodes
  std::vector<double> C;   // [nproc][n] cumulative frequency
  std::vector<double> P;   // [n] prefix maximum of the total frequency
  std::vector<double> node;
};

}  // namespace

extern "C" {

typedef struct orc_problem {
  double mass, charge, gas_N, target_mass;
  int n_e;
  double eps_min, eps_max;
  int n_proc;
  const int* kind;
  const double* threshold;
  const double* sigma;  // [n_proc][n_e]
  int flags;
} orc_problem;

typedef struct orc_grid {
  const double* E;  // [nz][ny][nx][3]
  int nx, ny, nz;
  double x0, y0, z0, dx;
} orc_grid;

}  // extern "C"

namespace {

// Collision-rate tables (Sec. 2.1.5): nu_k = N sigma_k v at log-spaced nodes,
// then cumulative sums in process order and the prefix maximum of the total.
int build_tables(const orc_problem* pb, Species& S, Tables& T) {
  if (!(pb->mass > 0) || pb->charge == 0 || !(pb->gas_N >= 0) || !(pb->target_mass > 0)) return -1;
  if (pb->n_e < 2 || !(pb->eps_min > 0) || !(pb->eps_max > pb->eps_min)) return -6;
  if (pb->n_proc < 1 || pb->n_proc > 8) return -6;
  S.m = pb->mass;
  S.q = pb->charge;
  S.N = pb->gas_N;
  S.M = pb->target_mass;
  S.k_eps = 0.5 * S.m / kEV;
  T.n = pb->n_e;
  T.nproc = pb->n_proc;
  T.lnmin = std::log(pb->eps_min);
  T.dlog = (std::log(pb->eps_max) - T.lnmin) / (T.n - 1);
  T.eps_max = pb->eps_max;
  T.kind.assign(pb->kind, pb->kind + T.nproc);
  T.thr.assign(pb->threshold, pb->threshold + T.nproc);
  for (int k = 0; k < T.nproc; ++k) {
    if (T.kind[k] < 0 || T.kind[k] > 3) return -6;
    if (!(T.thr[k] >= 0) || !std::isfinite(T.thr[k])) return -6;
  }
  T.node.resize(T.n);
  for (int i = 0; i < T.n; ++i) T.node[i] = std::exp(T.lnmin + i * T.dlog);
  std::vector<double> sig(pb->sigma, pb->sigma + (size_t)T.nproc * T.n);
  for (double s : sig)
    if (!(s >= 0) || !std::isfinite(s)) return -6;
  if (pb->flags & EFFECTIVE_TO_ELASTIC) {
    // Effective momentum-transfer -> elastic: subtract the inelastic sum
    // (Sec. 2.1.5); a negative difference is set to zero.
    for (int i = 0; i < T.n; ++i) {
      double inel = 0;
      for (int k = 0; k < T.nproc; ++k)
        if (T.kind[k] != ELASTIC) inel += sig[(size_t)k * T.n + i];
      for (int k = 0; k < T.nproc; ++k)
        if (T.kind[k] == ELASTIC) sig[(size_t)k * T.n + i] = std::max(0.0, sig[(size_t)k * T.n + i] - inel);
    }
  }
  T.nu.resize((size_t)T.nproc * T.n);
  for (int k = 0; k < T.nproc; ++k)
    for (int i = 0; i < T.n; ++i) {
      const double v = std::sqrt(2.0 * kEV * T.node[i] / S.m);
      const double s = sig[(size_t)k * T.n + i];
      T.nu[(size_t)k * T.n + i] = (pb->flags & RATES) ? s : S.N * s * v;
    }
  T.C.resize((size_t)T.nproc * T.n);
  for (int i = 0; i < T.n; ++i) {
    double acc = 0;
    for (int k = 0; k < T.nproc; ++k) {
      acc += T.nu[(size_t)k * T.n + i];
      T.C[(size_t)k * T.n + i] = acc;
    }
  }
  T.P.resize(T.n);
  double run = 0;
  for (int i = 0; i < T.n; ++i) {
    run = std::max(run, T.C[(size_t)(T.nproc - 1) * T.n + i]);
    T.P[i] = run;
  }
  return 0;
}

// Position in the table: interval i and fraction f, linear in ln(eps); rates
// are held constant outside the tabulated range.
void locate(const Tables& T, double eps, int& i, double& f) {
  double u = eps > 0 ? (std::log(eps) - T.lnmin) / T.dlog : -std::numeric_limits<double>::infinity();
  double fl = std::floor(u);
  if (!(fl >= 0)) fl = 0;
  if (fl > T.n - 2) fl = T.n - 2;
  i = (int)fl;
  f = u - fl;
  if (!(f >= 0)) f = 0;
  if (f > 1) f = 1;
}

double row_at(const Tables& T, const std::vector<double>& tab, int row, int i, double f) {
  const double* r = tab.data() + (size_t)row * T.n;
  return (1.0 - f) * r[i] + f * r[i + 1];
}

// Majorant of the total collision frequency for a particle whose speed stays
// below s_ub: the prefix maximum of the total rate, interpolated at the energy
// of s_ub (inflated by 2^-16 as a rounding guard), bounds the interpolated
// total rate at every lower energy.
double majorant(const Tables& T, const Species& S, double s_ub0) {
  const double s_ub = s_ub0 * (1.0 + 0x1p-16);
  const double eps_ub = S.k_eps * s_ub * s_ub;
  const double scale = g_majorant_fault == 2 ? 0.9 : 1.0;
  if (eps_ub >= T.node[T.n - 1]) return scale * T.P[T.n - 1];
  int i;
  double f;
  locate(T, eps_ub, i, f);
  return scale * ((1.0 - f) * T.P[i] + f * T.P[i + 1]);
}

struct Particle {
  double x[3], v[3], w;
  uint64_t id;
};

// The particle record holds single-precision position, velocity and weight
// (the particle arrays are single precision); within a step everything is
// computed in double precision and the record is rounded at the end of each
// step and when a newborn is queued.
void round_record(Particle& p) {
  for (int c = 0; c < 3; ++c) {
    p.x[c] = (double)(float)p.x[c];
    p.v[c] = (double)(float)p.v[c];
  }
}
struct Pending {
  Particle p;
  double tb;
};

// Bound on |a| along the rest of a step and on how much a can change there;
// local = taken from the particle's cell neighbourhood (not the global one).
struct ABound {
  double a_abs, da;
  bool local;
};

// Largest speed reachable within time h from velocity v under acceleration
// a0 now, if |a| <= b.a_abs and |a - a0| <= b.da along the way: the speed of
// v + a0 t is convex in t, so its maximum on [0, h] is at an end point.
double speed_bound(const double v[3], const double a0[3], double speed, const ABound& b, double h) {
  double w2 = 0;
  for (int c = 0; c < 3; ++c) {
    const double q = v[c] + a0[c] * h;
    w2 += q * q;
  }
  const double s_dir = std::max(speed, std::sqrt(w2)) + (g_majorant_fault == 1 ? 0.0 : b.da) * h;
  return std::min(speed + b.a_abs * h, s_dir);
}

// Event counters.  maj_viol counts flight segments whose end point has a
// total collision rate above the majorant the segment was drawn with (the
// null-collision method needs nu_hat >= nu_tot(eps) everywhere along the
// flight, Sec. 2.1.1; a count above zero means the bound is wrong);
// bound_local / bound_global count particle-steps whose field bound came from
// the 4x4x4 cell neighbourhood or from the global maximum.
struct Counters {
  int64_t trials = 0, null = 0, real[4] = {0, 0, 0, 0}, lost = 0, oot = 0, errors = 0;
  int64_t maj_viol = 0, bound_local = 0, bound_global = 0;
  void add(const Counters& o) {
    trials += o.trials;
    null += o.null;
    for (int k = 0; k < 4; ++k) real[k] += o.real[k];
    lost += o.lost;
    oot += o.oot;
    errors += o.errors;
    maj_viol += o.maj_viol;
    bound_local += o.bound_local;
    bound_global += o.bound_global;
  }
};

// Trilinear (CIC) field interpolation on cell centres (Sec. 2.1.3), indices
// clamped to the grid (constant extrapolation in the outer half cell).
struct GridAccel {
  const orc_grid* g;
  double qm;
  void operator()(const double x[3], double a[3]) const {
    const int n[3] = {g->nx, g->ny, g->nz};
    const double o[3] = {g->x0, g->y0, g->z0};
    int i0[3], i1[3];
    double wt[3][2];
    for (int d = 0; d < 3; ++d) {
      double u = (x[d] - o[d]) / g->dx - 0.5;
      if (u < -1) u = -1;
      if (u > n[d]) u = n[d];
      const double fl = std::floor(u);
      const double f = u - fl;
      const int i = (int)fl;
      i0[d] = std::min(std::max(i, 0), n[d] - 1);
      i1[d] = std::min(std::max(i + 1, 0), n[d] - 1);
      wt[d][0] = 1.0 - f;
      wt[d][1] = f;
    }
    double E[3] = {0, 0, 0};
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int ix = dx ? i1[0] : i0[0], iy = dy ? i1[1] : i0[1], iz = dz ? i1[2] : i0[2];
          const double W = wt[0][dx] * wt[1][dy] * wt[2][dz];
          const double* e = g->E + 3 * (((size_t)iz * g->ny + iy) * g->nx + ix);
          for (int c = 0; c < 3; ++c) E[c] += W * e[c];
        }
    for (int c = 0; c < 3; ++c) a[c] = qm * E[c];
  }

  // Bounds for the rest of a step of length t_rem.  The particle cannot be
  // faster than |v| + a_glob t along the way (collisions never add speed), so
  // it moves less than D = |v| t_rem + a_glob t_rem^2 / 2.  If D is below one
  // cell (with a 2^-10 margin), every position it reaches interpolates from
  // the 4x4x4 cell centres around its present cell; as trilinear
  // interpolation is a convex combination, |E| there is at most the largest
  // |E| of those centres (Amax) and two such fields differ by at most the
  // norm of their per-component ranges (Dvar).  Otherwise the global bound
  // a_glob is used, with |a - a0| <= 2 a_glob.
  const std::vector<double>* Amax;  // [nz][ny][nx]
  const std::vector<double>* Dvar;  // [nz][ny][nx]
  double a_glob;
  ABound bound(const Particle& p, double t_rem) const;
};

struct UniformAccel {
  double a[3];
  double a_abs;
  void operator()(const double*, double out[3]) const {
    out[0] = a[0];
    out[1] = a[1];
    out[2] = a[2];
  }
  ABound bound(const Particle&, double) const { return ABound{a_abs, 0.0, true}; }
};

ABound GridAccel::bound(const Particle& p, double t_rem) const {
  const double speed = std::sqrt(p.v[0] * p.v[0] + p.v[1] * p.v[1] + p.v[2] * p.v[2]);
  const double D = speed * t_rem + 0.5 * a_glob * t_rem * t_rem;
  if (!(D < g->dx * (1.0 - 0x1p-10))) return ABound{a_glob, 2.0 * a_glob, false};
  const int n[3] = {g->nx, g->ny, g->nz};
  const double o[3] = {g->x0, g->y0, g->z0};
  int b[3];
  for (int d = 0; d < 3; ++d) {
    double u = (p.x[d] - o[d]) / g->dx - 0.5;
    if (u < -1) u = -1;
    if (u > n[d]) u = n[d];
    b[d] = std::min(std::max((int)std::floor(u), 0), n[d] - 1);
  }
  const size_t c = ((size_t)b[2] * g->ny + b[1]) * g->nx + b[0];
  return ABound{std::fabs(qm) * (*Amax)[c], std::fabs(qm) * (*Dvar)[c], true};
}

// Advance one particle from time t0 to the end of the step (length dt):
// null-collision flight segments integrated with velocity Verlet, each ended
// by a real or a null collision.  Returns 0 if the particle is alive at the
// end of the step, 1 if it was attached, 2 if it hit the segment limit.
template <class Accel>
int advance(const Tables& T, const Species& S, const Accel& accel, Particle& p, double t0, double dt, uint32_t key0,
            uint32_t key1, uint64_t step, std::vector<Pending>& births, Counters& cnt) {
  double a[3];
  accel(p.x, a);
  double t = t0;
  const ABound bnd = accel.bound(p, dt - t0);  // fixed for this item's step
  (bnd.local ? cnt.bound_local : cnt.bound_global)++;
  // The majorant must bound the total rate wherever the flight reaches; it is
  // checked at the end point of every segment.
  auto check_majorant = [&](double nu_hat) {
    const double e = S.k_eps * (p.v[0] * p.v[0] + p.v[1] * p.v[1] + p.v[2] * p.v[2]);
    int ii;
    double ff;
    locate(T, e, ii, ff);
    if (row_at(T, T.C, T.nproc - 1, ii, ff) > nu_hat) cnt.maj_viol++;
  };
  // Velocity Verlet over a sub-interval h (eq. 1-2).
  auto verlet = [&](double h) {
    for (int c = 0; c < 3; ++c) p.x[c] += p.v[c] * h + 0.5 * a[c] * h * h;
    double an[3];
    accel(p.x, an);
    for (int c = 0; c < 3; ++c) {
      p.v[c] += 0.5 * (a[c] + an[c]) * h;
      a[c] = an[c];
    }
  };
  for (uint32_t j = 0;; ++j) {
    if (j >= (uint32_t)kMaxSegments) {
      cnt.errors++;
      return 2;
    }
    const Draw d = draw(key0, key1, p.id, step, j, TAG_MAIN);
    cnt.trials++;
    const double t_rem = dt - t;
    const double speed = std::sqrt(p.v[0] * p.v[0] + p.v[1] * p.v[1] + p.v[2] * p.v[2]);
    const double nu_full = g_constant_majorant ? T.P[T.n - 1] : majorant(T, S, speed_bound(p.v, a, speed, bnd, t_rem));
    const bool limited = !g_constant_majorant && KAPPA < nu_full * t_rem;
    const double h = limited ? KAPPA / nu_full : t_rem;
    const double nu_hat = limited ? majorant(T, S, speed_bound(p.v, a, speed, bnd, h)) : nu_full;
    const double tau = nu_hat > 0 ? -std::log(unif(d.r[0])) / nu_hat : std::numeric_limits<double>::infinity();
    if (tau >= h) {  // no candidate collision within the horizon
      verlet(h);
      check_majorant(nu_hat);
      if (!limited) return 0;
      t += h;
      continue;
    }
    verlet(tau);
    t += tau;
    check_majorant(nu_hat);
    const double v2 = p.v[0] * p.v[0] + p.v[1] * p.v[1] + p.v[2] * p.v[2];
    const double eps = S.k_eps * v2;
    int i;
    double f;
    locate(T, eps, i, f);
    const double y = unif(d.r[1]) * nu_hat;
    // Real or null: the first process whose cumulative rate exceeds y.
    int k = -1;
    for (int kk = 0; kk < T.nproc; ++kk)
      if (y < row_at(T, T.C, kk, i, f)) {
        k = kk;
        break;
      }
    if (k < 0 || eps < T.thr[k]) {  // null collision (also below threshold)
      cnt.null++;
      continue;
    }
    if (eps > T.eps_max) cnt.oot++;
    const int kind = T.kind[k];
    cnt.real[kind]++;
    if (kind == ATTACHMENT) return 1;
    // Isotropic new direction.
    const double cth = 1.0 - 2.0 * unif(d.r[2]);
    const double phi = 2.0 * kPI * unif(d.r[3]);
    const double sth = std::sqrt(std::max(0.0, 1.0 - cth * cth));
    const double n[3] = {sth * std::cos(phi), sth * std::sin(phi), cth};
    double eps_new;
    if (kind == ELASTIC) {
      // Elastic recoil against a cold heavy partner, to first order in m/M.
      const double speed_c = std::sqrt(v2);
      const double cchi = speed_c > 0 ? (p.v[0] * n[0] + p.v[1] * n[1] + p.v[2] * n[2]) / speed_c : 0.0;
      eps_new = eps * (1.0 - (2.0 * S.m / S.M) * (1.0 - cchi));
    } else if (kind == EXCITATION) {
      eps_new = eps - T.thr[k];
    } else {  // IONIZATION: the energy left after the threshold is shared equally.
      eps_new = 0.5 * (eps - T.thr[k]);
      const Draw b = draw(key0, key1, p.id, step, j, TAG_BIRTH);
      Pending c;
      c.p = p;
      c.p.id = (uint64_t)b.r[0] | ((uint64_t)b.r[1] << 32);
      const double ccth = 1.0 - 2.0 * unif(b.r[2]);
      const double cphi = 2.0 * kPI * unif(b.r[3]);
      const double csth = std::sqrt(std::max(0.0, 1.0 - ccth * ccth));
      const double cs = std::sqrt(eps_new / S.k_eps);
      c.p.v[0] = cs * csth * std::cos(cphi);
      c.p.v[1] = cs * csth * std::sin(cphi);
      c.p.v[2] = cs * ccth;
      round_record(c.p);
      c.tb = (double)(float)t;
      births.push_back(c);
    }
    const double s_new = std::sqrt(eps_new / S.k_eps);
    for (int c = 0; c < 3; ++c) p.v[c] = s_new * n[c];
  }
}

void set_threads(int n_threads) {
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
}

// A charge-creating event: where an ionization left its positive ion (the
// newborn's recorded position) or an attachment its negative ion (the
// electron's position at attachment, rounded to single precision), with the
// electron's weight.
struct Event {
  float x, y, z, w;
};

// One step of a particle population: every particle from t = 0, then the
// newborns from their birth times, generation after generation until none
// are left.  Survivors (alive and accepted by `keep`) are returned in `out`;
// ionization and attachment events are appended to ion_ev / att_ev if given.
template <class Accel, class Keep>
void run_step(const Tables& T, const Species& S, const Accel& accel, const std::vector<Particle>& in,
              double dt, uint32_t key0, uint32_t key1, uint64_t step, const Keep& keep, std::vector<Particle>& out,
              Counters& cnt, std::vector<Event>* ion_ev = nullptr, std::vector<Event>* att_ev = nullptr) {
  out.clear();
  std::vector<Pending> work(in.size());
  for (size_t i = 0; i < in.size(); ++i) work[i] = Pending{in[i], 0.0};
  while (!work.empty()) {
    std::vector<Pending> next_gen;
#pragma omp parallel
    {
      std::vector<Particle> my_out;
      std::vector<Pending> my_births;
      std::vector<Event> my_att;
      Counters my_cnt;
#pragma omp for schedule(static)
      for (int64_t i = 0; i < (int64_t)work.size(); ++i) {
        Particle p = work[i].p;
        const int r = advance(T, S, accel, p, work[i].tb, dt, key0, key1, step, my_births, my_cnt);
        if (r == 0) {
          if (keep(p)) {
            round_record(p);
            my_out.push_back(p);
          } else {
            my_cnt.lost++;
          }
        } else if (r == 1 && att_ev) {
          my_att.push_back(Event{(float)p.x[0], (float)p.x[1], (float)p.x[2], (float)p.w});
        }
      }
#pragma omp critical
      {
        out.insert(out.end(), my_out.begin(), my_out.end());
        next_gen.insert(next_gen.end(), my_births.begin(), my_births.end());
        if (ion_ev)
          for (const Pending& b : my_births)
            ion_ev->push_back(Event{(float)b.p.x[0], (float)b.p.x[1], (float)b.p.x[2], (float)b.p.w});
        if (att_ev) att_ev->insert(att_ev->end(), my_att.begin(), my_att.end());
        cnt.add(my_cnt);
      }
    }
    work.swap(next_gen);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Super-particle weights (Sec. 2.1.2).  The desired weight of cell c is
// omega_c = n_e dV / N_ppc with n_e dV the number of electrons the charge
// mapping puts on the cell (the CIC density, Sec. 2.1.3, in units of
// electrons) and omega_min = 1.  Particles in a cell with w < (2/3) omega are
// merged pairwise, pairs formed from particles close in energy; particles with
// w > (3/2) omega are split into two halves.  Readings where the paper is
// silent:
//   * the cell of a particle is the one containing it (floor of (x - x0)/dx,
//     clamped to the grid);
//   * "close in energy": the merge candidates of a cell are ordered by energy
//     (|v|^2 rounded to single precision), then by id, and consecutive ones
//     are paired; an odd one out stays as it is;
//   * the merged particle keeps the position, velocity and id of one of the
//     two, the first with probability w_a / (w_a + w_b) (so position and
//     momentum are conserved on average), drawn from the weight-update draw
//     of the smaller id; its weight is w_a + w_b;
//   * a split halves the weight once per update and adds a copy with the same
//     position and velocity; the copy's id is the (second, third) words of the
//     particle's weight-update draw;
//   * weight-update draws: counter (id, update index, 0, purpose 3).
struct WeightCounts {
  int64_t merged_pairs = 0, splits = 0;
};

int cell_of(double x, double o, double inv_dx, int n) {
  int i = (int)std::floor((x - o) * inv_dx);
  return std::min(std::max(i, 0), n - 1);
}

int update_weights(std::vector<Particle>& ps, int nx, int ny, int nz, double x0, double y0, double z0, double inv_dx,
                   double n_ppc, uint32_t key0, uint32_t key1, uint64_t update_index, WeightCounts& wc) {
  const size_t n = ps.size();
  const size_t ncell = (size_t)nx * ny * nz;
  std::vector<float> fx(n), fy(n), fz(n), fw(n);
  for (size_t i = 0; i < n; ++i) {
    fx[i] = (float)ps[i].x[0];
    fy[i] = (float)ps[i].x[1];
    fz[i] = (float)ps[i].x[2];
    fw[i] = (float)ps[i].w;
  }
  std::vector<int64_t> rho(ncell, 0);
  const int drc =
      orc_deposit_impl(fx.data(), fy.data(), fz.data(), fw.data(), (int64_t)n, nx, ny, nz, x0, y0, z0, inv_dx, rho.data());
  if (drc) return drc;
  std::vector<int64_t> cell(n);
  std::vector<int> cls(n, 0);  // 0 keep, 1 merge candidate, 2 split
  std::vector<size_t> cand;
  for (size_t i = 0; i < n; ++i) {
    const Particle& p = ps[i];
    const size_t c = ((size_t)cell_of(p.x[2], z0, inv_dx, nz) * ny + cell_of(p.x[1], y0, inv_dx, ny)) * nx +
                     cell_of(p.x[0], x0, inv_dx, nx);
    cell[i] = (int64_t)c;
    const double omega = std::max(std::ldexp((double)rho[c], -32) / n_ppc, 1.0);
    if (p.w < (2.0 / 3.0) * omega) {
      cls[i] = 1;
      cand.push_back(i);
    } else if (p.w > 1.5 * omega) {
      cls[i] = 2;
    }
  }
  auto ekey = [&](size_t i) {
    const Particle& p = ps[i];
    return (float)((p.v[0] * p.v[0] + p.v[1] * p.v[1]) + p.v[2] * p.v[2]);
  };
  std::sort(cand.begin(), cand.end(), [&](size_t a, size_t b) {
    if (cell[a] != cell[b]) return cell[a] < cell[b];
    const float ea = ekey(a), eb = ekey(b);
    if (ea != eb) return ea < eb;
    return ps[a].id < ps[b].id;
  });
  std::vector<char> removed(n, 0);
  size_t k = 0;
  while (k < cand.size()) {
    size_t e = k;
    while (e < cand.size() && cell[cand[e]] == cell[cand[k]]) ++e;
    for (size_t q = k; q + 1 < e; q += 2) {
      Particle& a = ps[cand[q]];
      Particle& b = ps[cand[q + 1]];
      const Draw d = draw(key0, key1, std::min(a.id, b.id), update_index, 0, TAG_WEIGHT);
      const double pa = a.w / (a.w + b.w);
      const double wsum = (double)(float)(a.w + b.w);
      if (unif(d.r[0]) < pa) {
        a.w = wsum;
        removed[cand[q + 1]] = 1;
      } else {
        b.w = wsum;
        removed[cand[q]] = 1;
      }
      ++wc.merged_pairs;
    }
    k = e;
  }
  std::vector<Particle> out;
  out.reserve(n + n / 4);
  std::vector<Particle> copies;
  for (size_t i = 0; i < n; ++i) {
    if (removed[i]) continue;
    Particle p = ps[i];
    if (cls[i] == 2) {
      p.w = 0.5 * p.w;
      const Draw d = draw(key0, key1, p.id, update_index, 0, TAG_WEIGHT);
      Particle c = p;
      c.id = (uint64_t)d.r[1] | ((uint64_t)d.r[2] << 32);
      copies.push_back(c);
      ++wc.splits;
    }
    out.push_back(p);
  }
  out.insert(out.end(), copies.begin(), copies.end());
  ps.swap(out);
  return 0;
}

extern "C" {

void orc_set_constant_majorant(int on) { g_constant_majorant = on; }
void orc_set_majorant_fault(int mode) { g_majorant_fault = mode; }

void orc_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) {
    uint32_t c[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
    philox4x32_10(c, key[2 * i], key[2 * i + 1]);
    std::memcpy(out + 4 * i, c, sizeof(c));
  }
}

// Exposes the tables for the tests: node energies [n_e], per-process rates
// [n_proc][n_e], cumulative rates [n_proc][n_e] and the prefix maximum [n_e].
int orc_build_tables(const orc_problem* pb, double* node, double* nu, double* C, double* P) {
  Species S;
  Tables T;
  const int rc = build_tables(pb, S, T);
  if (rc) return rc;
  std::copy(T.node.begin(), T.node.end(), node);
  std::copy(T.nu.begin(), T.nu.end(), nu);
  std::copy(T.C.begin(), T.C.end(), C);
  std::copy(T.P.begin(), T.P.end(), P);
  return 0;
}

// Table lookups at arbitrary energies (tests): interpolated cumulative rates
// [m][n_proc] and the majorant for given speed bounds s_ub[m].
int orc_lookup(const orc_problem* pb, int64_t m, const double* eps, double* C_out, const double* s_ub,
               double* maj_out) {
  Species S;
  Tables T;
  const int rc = build_tables(pb, S, T);
  if (rc) return rc;
  for (int64_t q = 0; q < m; ++q) {
    int i;
    double f;
    locate(T, eps[q], i, f);
    for (int k = 0; k < T.nproc; ++k) C_out[q * T.nproc + k] = row_at(T, T.C, k, i, f);
    if (maj_out) maj_out[q] = majorant(T, S, s_ub[q]);
  }
  return 0;
}

// PIC-MCC electron update over n_steps steps of a fixed field (the state is
// in double precision; arrays have room for `capacity` particles).  Stats
// layout: n, steps_done, particle_steps, trials, null, elastic, excitation,
// ionization, attachment, lost, out_of_table, errors.
// Weight control (n_ppc > 0): after a committed step s, if the particle count
// exceeds floor(growth * n_ref), the weights are updated with update index
// step0 + s and n_ref becomes the new count; n_ref (in/out) starts at the
// count of the first call when 0.  wstats (nullable) receives the number of
// updates, merged pairs and splits.
int orc_pic_run(const orc_problem* pb, const orc_grid* g, double* x, double* y, double* z, double* vx, double* vy,
                double* vz, double* w, uint64_t* id, int64_t* n_inout, int64_t capacity, double dt, int n_steps,
                uint64_t seed, uint64_t step0, int64_t* stats, int n_threads, double n_ppc, double growth,
                int64_t* n_ref, int64_t* wstats, float* ion_ev, float* att_ev, int64_t ev_cap, int64_t* ev_counts) {
  Species S;
  Tables T;
  int rc = build_tables(pb, S, T);
  if (rc) return rc;
  if (!g || !g->E || g->nx < 1 || g->ny < 1 || g->nz < 1 || !(g->dx > 0)) return -1;
  if (*n_inout < 0 || *n_inout > capacity || !(dt > 0) || n_steps < 0) return -1;
  set_threads(n_threads);
  double emax = 0;
  const size_t ncell = (size_t)g->nx * g->ny * g->nz;
  std::vector<double> Emag(ncell), Amax(ncell), Dvar(ncell);
  for (size_t c = 0; c < ncell; ++c) {
    const double* e = g->E + 3 * c;
    Emag[c] = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    emax = std::max(emax, Emag[c]);
  }
#pragma omp parallel for schedule(static)
  for (int k = 0; k < g->nz; ++k)
    for (int j = 0; j < g->ny; ++j)
      for (int i = 0; i < g->nx; ++i) {
        double m = 0, lo[3], hi[3];
        for (int q = 0; q < 3; ++q) {
          lo[q] = std::numeric_limits<double>::infinity();
          hi[q] = -std::numeric_limits<double>::infinity();
        }
        for (int kk = std::max(k - 1, 0); kk <= std::min(k + 2, g->nz - 1); ++kk)
          for (int jj = std::max(j - 1, 0); jj <= std::min(j + 2, g->ny - 1); ++jj)
            for (int ii = std::max(i - 1, 0); ii <= std::min(i + 2, g->nx - 1); ++ii) {
              const size_t cc = ((size_t)kk * g->ny + jj) * g->nx + ii;
              m = std::max(m, Emag[cc]);
              for (int q = 0; q < 3; ++q) {
                lo[q] = std::min(lo[q], g->E[3 * cc + q]);
                hi[q] = std::max(hi[q], g->E[3 * cc + q]);
              }
            }
        const size_t c = ((size_t)k * g->ny + j) * g->nx + i;
        Amax[c] = m;
        Dvar[c] = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                            (hi[2] - lo[2]) * (hi[2] - lo[2]));
      }
  GridAccel accel{g, S.q / S.m, &Amax, &Dvar, std::fabs(S.q / S.m) * emax};
  const double lo[3] = {g->x0, g->y0, g->z0};
  const double hi[3] = {g->x0 + g->nx * g->dx, g->y0 + g->ny * g->dx, g->z0 + g->nz * g->dx};
  auto inside = [&](const Particle& p) {
    for (int c = 0; c < 3; ++c)
      if (!(p.x[c] >= lo[c] && p.x[c] < hi[c])) return false;
    return true;
  };
  std::vector<Particle> cur((size_t)*n_inout), nxt;
  for (int64_t i = 0; i < *n_inout; ++i) {
    Particle& p = cur[i];
    p.x[0] = x[i];
    p.x[1] = y[i];
    p.x[2] = z[i];
    p.v[0] = vx[i];
    p.v[1] = vy[i];
    p.v[2] = vz[i];
    p.w = (double)(float)w[i];
    p.id = id[i];
    round_record(p);
  }
  Counters total;
  int64_t steps_done = 0, particle_steps = 0;
  const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
  WeightCounts wc;
  int64_t updates = 0;
  int64_t nref = n_ref && *n_ref > 0 ? *n_ref : (int64_t)cur.size();
  rc = 0;
  const bool events = ion_ev && att_ev && ev_counts;
  std::vector<Event> ions, atts, step_ions, step_atts;
  for (int s = 0; s < n_steps; ++s) {
    Counters cnt;
    step_ions.clear();
    step_atts.clear();
    run_step(T, S, accel, cur, dt, key0, key1, step0 + s, inside, nxt, cnt, events ? &step_ions : nullptr,
             events ? &step_atts : nullptr);
    if ((int64_t)nxt.size() > capacity) {
      rc = -2;
      break;
    }
    ions.insert(ions.end(), step_ions.begin(), step_ions.end());
    atts.insert(atts.end(), step_atts.begin(), step_atts.end());
    particle_steps += (int64_t)cur.size();
    cur.swap(nxt);
    total.add(cnt);
    ++steps_done;
    if (n_ppc > 0 && (int64_t)cur.size() > (int64_t)std::floor(growth * (double)nref)) {
      const int urc =
          update_weights(cur, g->nx, g->ny, g->nz, g->x0, g->y0, g->z0, 1.0 / g->dx, n_ppc, key0, key1, step0 + s, wc);
      if (urc) {
        rc = urc;
        break;
      }
      if ((int64_t)cur.size() > capacity) {
        rc = -2;
        break;
      }
      nref = (int64_t)cur.size();
      ++updates;
    }
  }
  if (n_ref) *n_ref = nref;
  if (events) {
    ev_counts[0] = (int64_t)ions.size();
    ev_counts[1] = (int64_t)atts.size();
    if ((int64_t)ions.size() > ev_cap || (int64_t)atts.size() > ev_cap) {
      if (rc == 0) rc = -2;
    } else {
      std::memcpy(ion_ev, ions.data(), ions.size() * sizeof(Event));
      std::memcpy(att_ev, atts.data(), atts.size() * sizeof(Event));
    }
  }
  if (wstats) {
    wstats[0] = updates;
    wstats[1] = wc.merged_pairs;
    wstats[2] = wc.splits;
  }
  for (size_t i = 0; i < cur.size(); ++i) {
    const Particle& p = cur[i];
    x[i] = p.x[0];
    y[i] = p.x[1];
    z[i] = p.x[2];
    vx[i] = p.v[0];
    vy[i] = p.v[1];
    vz[i] = p.v[2];
    w[i] = p.w;
    id[i] = p.id;
  }
  *n_inout = (int64_t)cur.size();
  if (stats) {
    const int64_t v[15] = {(int64_t)cur.size(), steps_done,    particle_steps, total.trials,
                           total.null,          total.real[0], total.real[1],  total.real[2],
                           total.real[3],       total.lost,    total.oot,      total.errors,
                           total.maj_viol,      total.bound_local, total.bound_global};
    std::memcpy(stats, v, sizeof(v));
  }
  return rc;
}

// CIC deposit (Sec. 2.1.3) in 2^-32 fixed point on identical single-precision
// particle arrays.  Per axis u = (x - x0) * inv_dx - 1/2, cell i = floor(u),
// weights (1 - f, f); corners visited in (dz, dy, dx) order, each rounded to
// the nearest integer, the last corner taking the remainder so the particle's
// charge w * 2^32 is conserved exactly.  Indices are clamped (folded back).
// Returns ORC_ERANGE (rho unchanged) for a weight outside [0, 2^31) or a cell
// whose exact sum leaves the int64 range (2^31 electrons per cell).
int orc_deposit(const float* x, const float* y, const float* z, const float* w, int64_t n, int nx, int ny, int nz,
                double x0, double y0, double z0, double inv_dx, int64_t* rho) {
  return orc_deposit_impl(x, y, z, w, n, nx, ny, nz, x0, y0, z0, inv_dx, rho);
}

}  // extern "C"

int orc_deposit_impl(const float* x, const float* y, const float* z, const float* w, int64_t n, int nx, int ny,
                     int nz, double x0, double y0, double z0, double inv_dx, int64_t* rho) {
  const int nn[3] = {nx, ny, nz};
  const double o[3] = {x0, y0, z0};
  // a particle's charge round(w 2^32) must fit one corner: 0 <= w < 2^31
  for (int64_t p = 0; p < n; ++p)
    if (!((double)w[p] >= 0.0 && (double)w[p] < 2147483648.0)) return ORC_ERANGE;
  // exact cell sums (128-bit), stored only if every one fits int64
  const size_t ncell = (size_t)nx * ny * nz;
  std::vector<__int128> acc(rho, rho + ncell);
  for (int64_t p = 0; p < n; ++p) {
    const double pos[3] = {(double)x[p], (double)y[p], (double)z[p]};
    const double wd = (double)w[p];
    const int64_t qw = std::llrint(std::ldexp(wd, 32));
    int ic[3][2];
    double W[3][2];
    for (int d = 0; d < 3; ++d) {
      double u = (pos[d] - o[d]) * inv_dx - 0.5;
      if (u < -1) u = -1;
      if (u > nn[d]) u = nn[d];
      const double fl = std::floor(u);
      const double f = u - fl;
      const int i = (int)fl;
      ic[d][0] = std::min(std::max(i, 0), nn[d] - 1);
      ic[d][1] = std::min(std::max(i + 1, 0), nn[d] - 1);
      W[d][0] = 1.0 - f;
      W[d][1] = f;
    }
    int64_t given = 0;
    for (int dz = 0; dz < 2; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          int64_t c;
          if (dz & dy & dx) {
            c = qw - given;
          } else {
            const double frac = (W[0][dx] * W[1][dy]) * W[2][dz];
            c = std::llrint(std::ldexp(wd * frac, 32));
            given += c;
          }
          const size_t cell = ((size_t)ic[2][dz] * ny + ic[1][dy]) * nx + ic[0][dx];
          acc[cell] += c;
        }
  }
  for (size_t c = 0; c < ncell; ++c)
    if (acc[c] > (__int128)INT64_MAX || acc[c] < (__int128)INT64_MIN) return ORC_ERANGE;
  for (size_t c = 0; c < ncell; ++c) rho[c] = (int64_t)acc[c];
  return 0;
}

extern "C" {

// Uniform-field swarms (Sec. 2.2.2): swarm s starts with n0[s] electrons at
// rest at the origin in a field E = (E/N) N along +z and is advanced n_steps
// steps.  Every `sample_every` steps the moments of the population (after the
// step's newborns, before population control) are recorded:
//   moments[s][j][14] = count, Sx, Sy, Sz, S(x^2+y^2), Sz^2, Svx, Svy, Svz,
//                       S(x vx + y vy), S(z vz), S eps, S nu_ion(eps), S nu_att(eps)
//   counters[s][j][4] = live count, log2 weight scale L, cumulative
//                       ionizations, cumulative attachments.
// Population control after each step (if pop_control): above 2 n0 every particle is kept with
// probability 2^-k (the smallest k that brings the expected count to 2 n0 or
// below) and L += k; below n0/2 every particle is duplicated and L -= 1.
int orc_swarm_run(const orc_problem* pb, int n_swarms, const double* EN_Td, const int32_t* n0, double dt,
                  int n_steps, uint64_t seed, int sample_every, int64_t cap_factor, int pop_control, double* moments,
                  int64_t* counters, int64_t* stats, int n_threads) {
  Species S;
  Tables T;
  int rc = build_tables(pb, S, T);
  if (rc) return rc;
  if (n_swarms < 1 || !(dt > 0) || n_steps < 0 || sample_every < 1 || cap_factor < 1) return -1;
  set_threads(n_threads);
  const int n_samples = n_steps / sample_every;
  int err = 0;
  Counters grand;
  int64_t grand_psteps = 0;
  for (int sw = 0; sw < n_swarms; ++sw) {
    if (n0[sw] < 1) return -1;
    const double E = EN_Td[sw] * 1e-21 * S.N;
    UniformAccel accel{{0.0, 0.0, (S.q / S.m) * E}, std::fabs(S.q / S.m) * E};
    const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32) ^ (uint32_t)sw;
    std::vector<Particle> cur(n0[sw]), nxt;
    for (int i = 0; i < n0[sw]; ++i) {
      Particle& p = cur[i];
      std::memset(&p, 0, sizeof(p));
      p.w = 1.0;
      p.id = (uint64_t)i;
    }
    int64_t L = 0, cum_ion = 0, cum_att = 0;
    const int64_t cap = cap_factor * (int64_t)n0[sw];
    for (int s = 0; s < n_steps; ++s) {
      Counters cnt;
      auto keep_all = [](const Particle&) { return true; };
      run_step(T, S, accel, cur, dt, key0, key1, (uint64_t)s, keep_all, nxt, cnt);
      if ((int64_t)nxt.size() > cap) {
        err = -2;
        break;
      }
      grand_psteps += (int64_t)cur.size();
      cur.swap(nxt);
      grand.add(cnt);
      cum_ion += cnt.real[IONIZATION];
      cum_att += cnt.real[ATTACHMENT];
      if ((s + 1) % sample_every == 0 && (s + 1) / sample_every <= n_samples) {
        const int jdx = (s + 1) / sample_every - 1;
        double m[14] = {0};
        for (const Particle& p : cur) {
          const double v2 = p.v[0] * p.v[0] + p.v[1] * p.v[1] + p.v[2] * p.v[2];
          const double eps = S.k_eps * v2;
          int i;
          double f;
          locate(T, eps, i, f);
          double nu_ion = 0, nu_att = 0;
          for (int k = 0; k < T.nproc; ++k) {
            if (eps < T.thr[k]) continue;
            const double nk = row_at(T, T.nu, k, i, f);
            if (T.kind[k] == IONIZATION) nu_ion += nk;
            if (T.kind[k] == ATTACHMENT) nu_att += nk;
          }
          m[0] += 1;
          m[1] += p.x[0];
          m[2] += p.x[1];
          m[3] += p.x[2];
          m[4] += p.x[0] * p.x[0] + p.x[1] * p.x[1];
          m[5] += p.x[2] * p.x[2];
          m[6] += p.v[0];
          m[7] += p.v[1];
          m[8] += p.v[2];
          m[9] += p.x[0] * p.v[0] + p.x[1] * p.v[1];
          m[10] += p.x[2] * p.v[2];
          m[11] += eps;
          m[12] += nu_ion;
          m[13] += nu_att;
        }
        std::memcpy(moments + ((size_t)sw * n_samples + jdx) * 14, m, sizeof(m));
        int64_t* cc = counters + ((size_t)sw * n_samples + jdx) * 4;
        cc[0] = (int64_t)cur.size();
        cc[1] = L;
        cc[2] = cum_ion;
        cc[3] = cum_att;
      }
      // Population control.
      const int64_t N = (int64_t)cur.size();
      const int64_t n0s = n0[sw];
      if (!pop_control) {
        // off: the population is left as it is
      } else if (N > 2 * n0s) {
        int k = 1;
        while (std::ldexp((double)N, -k) > 2.0 * (double)n0s) ++k;
        const double p_keep = std::ldexp(1.0, -k);
        nxt.clear();
        for (const Particle& p : cur) {
          const Draw d = draw(key0, key1, p.id, (uint64_t)s, 0, TAG_AUX);
          if (unif(d.r[0]) < p_keep) nxt.push_back(p);
        }
        cur.swap(nxt);
        L += k;
      } else if (N > 0 && 2 * N < n0s) {
        const size_t n_old = cur.size();
        for (size_t i = 0; i < n_old; ++i) {
          Particle dup = cur[i];
          const Draw d = draw(key0, key1, dup.id, (uint64_t)s, 0, TAG_AUX);
          dup.id = (uint64_t)d.r[1] | ((uint64_t)d.r[2] << 32);
          cur.push_back(dup);
        }
        L -= 1;
      }
    }
    if (err) break;
  }
  if (stats) {
    const int64_t v[15] = {0,           n_steps,       grand_psteps,  grand.trials,  grand.null, grand.real[0],
                           grand.real[1], grand.real[2], grand.real[3], grand.lost, grand.oot,  grand.errors,
                           grand.maj_viol, grand.bound_local, grand.bound_global};
    std::memcpy(stats, v, sizeof(v));
  }
  return err;
}

// Weight update of n particles (single-precision arrays) on the grid
// (nx, ny, nz, x0, y0, z0, dx); the result (at most `capacity` particles,
// input order with removed particles dropped, split copies appended) goes to
// the *_out arrays.  counts (nullable) = merged pairs, splits.  Returns -2
// when the result exceeds the capacity.
int orc_update_weights(const float* x, const float* y, const float* z, const float* vx, const float* vy,
                       const float* vz, const float* w, const uint64_t* id, int64_t n, int nx, int ny, int nz, double x0,
                       double y0, double z0, double dx, double n_ppc, uint64_t seed, uint64_t update_index,
                       float* x_out, float* y_out, float* z_out, float* vx_out, float* vy_out, float* vz_out,
                       float* w_out, uint64_t* id_out, int64_t capacity, int64_t* n_out, int64_t* counts) {
  if (n < 0 || nx < 1 || ny < 1 || nz < 1 || !(dx > 0) || !(n_ppc > 0)) return -1;
  std::vector<Particle> ps((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    ps[i].x[0] = x[i];
    ps[i].x[1] = y[i];
    ps[i].x[2] = z[i];
    ps[i].v[0] = vx[i];
    ps[i].v[1] = vy[i];
    ps[i].v[2] = vz[i];
    ps[i].w = w[i];
    ps[i].id = id[i];
  }
  WeightCounts wc;
  const int urc = update_weights(ps, nx, ny, nz, x0, y0, z0, 1.0 / dx, n_ppc, (uint32_t)seed, (uint32_t)(seed >> 32),
                                 update_index, wc);
  if (urc) return urc;
  if (counts) {
    counts[0] = wc.merged_pairs;
    counts[1] = wc.splits;
  }
  *n_out = (int64_t)ps.size();
  if ((int64_t)ps.size() > capacity) return -2;
  for (size_t i = 0; i < ps.size(); ++i) {
    x_out[i] = (float)ps[i].x[0];
    y_out[i] = (float)ps[i].x[1];
    z_out[i] = (float)ps[i].x[2];
    vx_out[i] = (float)ps[i].v[0];
    vy_out[i] = (float)ps[i].v[1];
    vz_out[i] = (float)ps[i].v[2];
    w_out[i] = (float)ps[i].w;
    id_out[i] = ps[i].id;
  }
  return 0;
}

}  // extern "C"
