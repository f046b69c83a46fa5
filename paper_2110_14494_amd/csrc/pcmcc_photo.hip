// Discrete photoionization (arXiv:2110.14494 Sec. 2.4: Zheleznyak's model,
// photons produced in proportion to the ionizations by the eq. of the UV
// source term, isotropic directions, absorption function f(r), simulated with
// discrete photons).
//
// * lambda = eta w / w_photon photons per ionization event of weight w
//   (w_photon <= 0: photons of the event's weight, lambda = eta); the count
//   is floor(lambda) plus one with probability lambda - floor(lambda).
// * Absorption distance: F(r) = U with F(r) = 1 - (E1(k1 r) - E1(k2 r)) /
//   ln(k2 / k1), the distribution function of f(r) = (exp(-k1 r) -
//   exp(-k2 r)) / (r ln(k2 / k1)) (the tail integral of (exp(-a s) -
//   exp(-b s)) / s from r to infinity is E1(a r) - E1(b r)); solved on ln r
//   by safeguarded Newton steps.
// * Draws: Philox4x32-10 keyed by the run seed and the step, counter = the
//   event's position bits and a word per purpose, so the photons of an event
//   do not depend on where the event sits in the list.
// Photons are rare (a few per thousand ionizations) and each is a long
// serial FP64 chain (the root of F): the counts of all events are scanned so
// that every photon gets a thread of its own, and all chains run at once.
#include <hip/hip_runtime.h>

#include <cstring>
#include <rocprim/rocprim.hpp>

#include "pcmcc_photo.hpp"

namespace pcmcc {

namespace {

// Exponential integral E1(x), x > 0: the power series -gamma - ln x -
// sum_k (-x)^k / (k k!) for x <= 2 (Abramowitz & Stegun 5.1.11; its
// cancellation costs about 1e-15 absolute at x = 2), else the continued
// fraction e^-x / (x + 1 - 1 / (x + 3 - 4 / (x + 5 - ...))) (A&S 5.1.22) by
// the modified Lentz method (at most about 46 terms from x = 2 on).
__device__ double e1(double x) {
  if (x <= 2.0) {
    double term = 1.0, sum = 0.0;
    for (int k = 1; k <= 60; ++k) {
      term *= -x / (double)k;  // (-x)^k / k!
      const double add = term / (double)k;
      sum += add;
      if (fabs(add) <= 1e-18) break;
    }
    return -0.57721566490153286061 - log(x) - sum;
  }
  if (x > 740.0) return 0.0;
  const double tiny = 1e-300;
  double b = x + 1.0, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i <= 300; ++i) {
    const double a = -(double)i * (double)i;
    b += 2.0;
    d = a * d + b;
    d = 1.0 / (fabs(d) < tiny ? tiny : d);
    c = b + a / c;
    if (fabs(c) < tiny) c = tiny;
    const double del = c * d;
    h *= del;
    if (fabs(del - 1.0) <= 1e-15) break;  // (a test below one ulp of 1 would never end the loop)
  }
  return h * exp(-x);
}

__device__ __forceinline__ double absorb_cdf(const PhotoArgs& A, double r) {
  return 1.0 - (e1(A.k1 * r) - e1(A.k2 * r)) / A.ln_k;
}

// r with F(r) = U: safeguarded Newton steps on s = ln r (dF/ds = (exp(-k1 r)
// - exp(-k2 r)) / ln(k2 / k1)), a bisection of the bracket whenever a step
// would leave it, from the geometric-mean absorption length; the bracket
// starts as [s_lo, s_hi].  Stops when |F - U| <= 2^-52 (F's own accuracy) or
// a step moves s by at most 1e-14.
__device__ double absorb_distance(const PhotoArgs& A, double U) {
  double lo = A.s_lo, hi = A.s_hi;
  double s = fmin(fmax(-0.5 * log(A.k1 * A.k2), lo), hi);
  for (int it = 0; it < 200; ++it) {
    const double r = exp(s);
    const double g = absorb_cdf(A, r) - U;
    if (fabs(g) <= 0x1p-52) break;
    if (g < 0.0) lo = s;
    else hi = s;
    const double dF = (exp(-A.k1 * r) - exp(-A.k2 * r)) / A.ln_k;
    double sn = s - g / dF;
    if (!(dF > 0.0) || !(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
    const double step = fabs(sn - s);
    s = sn;
    if (step <= 1e-14 || hi - lo <= 1e-14) break;
  }
  return exp(s);
}

__device__ __forceinline__ uint4 photo_draw(const PhotoArgs& A, uint32_t xb, uint32_t yb, uint32_t zb, uint32_t c) {
  return philox(make_uint4(xb, yb, zb, c), A.key);
}

__device__ __forceinline__ double u32(uint32_t r) { return ((double)r + 0.5) * 0x1p-32; }

__device__ __forceinline__ uint32_t photon_count(const PhotoArgs& A, uint64_t e, uint32_t& xb, uint32_t& yb,
                                                 uint32_t& zb, double& wph) {
#pragma clang fp contract(off)
  const float w = A.ew[e];
  xb = __float_as_uint(A.ex[e]);
  yb = __float_as_uint(A.ey[e]);
  zb = __float_as_uint(A.ez[e]);
  double lam;
  if (A.w_ph > 0.0) {
    lam = A.eta * (double)w / A.w_ph;
    wph = A.w_ph;
  } else {
    lam = A.eta;
    wph = (double)w;
  }
  if (!(lam > 0.0)) return 0u;
  if (lam >= 2147483648.0) return 0x80000000u;  // saturated: far beyond any particle capacity
  const double fl = floor(lam);
  const uint4 r = photo_draw(A, xb, yb, zb, 0u);
  return (uint32_t)fl + (u32(r.x) < lam - fl ? 1u : 0u);
}

}  // namespace

// Photon count of every event.
__global__ __launch_bounds__(256) void k_ph_count(PhotoArgs A, uint32_t* __restrict__ counts) {
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < A.n; e += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t xb, yb, zb;
    double wph;
    counts[e] = photon_count(A, e, xb, yb, zb, wph);
  }
}

// One thread per photon p < total: its event is the last e with offs[e] <=
// p (offs the exclusive scan of the counts), its index j = p - offs[e];
// direction, distance, absorption point; the photoelectrons absorbed inside
// the box are appended at *n_dev, one atomic per wave.
__global__ __launch_bounds__(256) void k_ph_emit(PhotoArgs A) {
#pragma clang fp contract(off)
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool keep = false;
  float px = 0.0f, py = 0.0f, pz = 0.0f, pw = 0.0f;
  uint64_t id = 0;
  if (p < A.total) {
    uint64_t lo = 0, hi = A.n;  // offs[lo] <= p < offs[hi], offs[n] = total
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (A.offs[mid] <= p) lo = mid;
      else hi = mid;
    }
    const uint64_t e = lo;
    const uint32_t j = (uint32_t)(p - A.offs[e]);
    const uint32_t xb = __float_as_uint(A.ex[e]), yb = __float_as_uint(A.ey[e]), zb = __float_as_uint(A.ez[e]);
    pw = A.w_ph > 0.0 ? (float)A.w_ph : A.ew[e];
    const uint4 r = photo_draw(A, xb, yb, zb, 2u * j + 1u);
    const double ct = 1.0 - 2.0 * u32(r.x);
    const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    const double ph = 6.283185307179586477 * u32(r.y);
    double sp, cp;
    sincos(ph, &sp, &cp);
    const double U = ((double)(r.z >> 5) * 67108864.0 + (double)(r.w >> 6) + 0.5) * 0x1p-53;
    const double dist = absorb_distance(A, U);
    px = (float)((double)__uint_as_float(xb) + dist * (st * cp));
    py = (float)((double)__uint_as_float(yb) + dist * (st * sp));
    pz = (float)((double)__uint_as_float(zb) + dist * ct);
    keep = (double)px >= A.lo[0] && (double)px < A.hi[0] && (double)py >= A.lo[1] && (double)py < A.hi[1] &&
           (double)pz >= A.lo[2] && (double)pz < A.hi[2];
    const uint4 q = photo_draw(A, xb, yb, zb, 2u * j + 2u);
    id = (uint64_t)q.x | ((uint64_t)q.y << 32);
  }
  const uint64_t m = __ballot(keep);
  if (m == 0) return;
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if ((int)lane == leader) base = atomicAdd(A.n_dev, (unsigned long long)__popcll(m));
  const uint32_t blo = __builtin_amdgcn_readlane((uint32_t)base, leader);
  const uint32_t bhi = __builtin_amdgcn_readlane((uint32_t)(base >> 32), leader);
  if (keep) {
    const uint64_t slot = (((uint64_t)bhi << 32) | blo) + (uint64_t)__popcll(m & ((1ull << lane) - 1ull));
    A.x[slot] = px;
    A.y[slot] = py;
    A.z[slot] = pz;
    A.vx[slot] = 0.0f;
    A.vy[slot] = 0.0f;
    A.vz[slot] = 0.0f;
    A.w[slot] = pw;
    A.id[slot] = id;
  }
}

static unsigned ph_blocks(uint64_t n) {
  const uint64_t b = (n + 255) / 256;
  return (unsigned)(b < 1024 ? (b > 0 ? b : 1) : 1024);
}

hipError_t photo_scan_bytes(uint64_t n, size_t* bytes) {
  return rocprim::exclusive_scan(nullptr, *bytes, (const uint32_t*)nullptr, (uint64_t*)nullptr, (uint64_t)0,
                                 (size_t)n, rocprim::plus<uint64_t>());
}

hipError_t launch_photo_count(const PhotoArgs& A, uint32_t* counts, void* temp, size_t temp_bytes, uint64_t* offs,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_ph_count, dim3(ph_blocks(A.n)), dim3(256), 0, s, A, counts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return rocprim::exclusive_scan(temp, temp_bytes, (const uint32_t*)counts, offs, (uint64_t)0, (size_t)A.n,
                                 rocprim::plus<uint64_t>(), s);
}

hipError_t launch_photo_emit(const PhotoArgs& A, hipStream_t s) {
  if (A.total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ph_emit, dim3((unsigned)((A.total + 255) / 256)), dim3(256), 0, s, A);
  return hipGetLastError();
}

}  // namespace pcmcc
