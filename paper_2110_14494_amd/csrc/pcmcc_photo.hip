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
//   exp(-b s)) / s from r to infinity is E1(a r) - E1(b r)); solved by 64
//   bisections on ln r.
// * Draws: Philox4x32-10 keyed by the run seed and the step, counter = the
//   event's position bits and a word per purpose, so the photons of an event
//   do not depend on where the event sits in the list.
// Work is tiny next to the particle step (a few photons per thousand
// ionizations): one thread per event, a wave-uniform loop over the photons,
// one append atomic per wave and photon round.
#include <hip/hip_runtime.h>

#include "pcmcc_photo.hpp"

namespace pcmcc {

namespace {

// Exponential integral E1(x), x > 0: the power series -gamma - ln x -
// sum_k (-x)^k / (k k!) for x <= 1 (Abramowitz & Stegun 5.1.11), else the
// continued fraction e^-x / (x + 1 - 1 / (x + 3 - 4 / (x + 5 - ...)))
// (A&S 5.1.22) by the modified Lentz method.
__device__ double e1(double x) {
  if (x <= 1.0) {
    double term = 1.0, sum = 0.0;
    for (int k = 1; k <= 40; ++k) {
      term *= -x / (double)k;  // (-x)^k / k!
      sum += term / (double)k;
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
    if (fabs(del - 1.0) < 1e-16) break;
  }
  return h * exp(-x);
}

__device__ __forceinline__ double absorb_cdf(const PhotoArgs& A, double r) {
  return 1.0 - (e1(A.k1 * r) - e1(A.k2 * r)) / A.ln_k;
}

// r with F(r) = U: 64 bisections on ln r over [s_lo, s_hi].
__device__ double absorb_distance(const PhotoArgs& A, double U) {
  double lo = A.s_lo, hi = A.s_hi;
  for (int it = 0; it < 64; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (absorb_cdf(A, exp(mid)) < U) lo = mid;
    else hi = mid;
  }
  return exp(0.5 * (lo + hi));
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
  const double fl = floor(lam);
  const uint4 r = photo_draw(A, xb, yb, zb, 0u);
  return (uint32_t)fl + (u32(r.x) < lam - fl ? 1u : 0u);
}

}  // namespace

// Photons emitted by the events: one atomic per block.
__global__ __launch_bounds__(256) void k_ph_count(PhotoArgs A, unsigned long long* total) {
  __shared__ unsigned long long s_w[4];
  unsigned long long m = 0;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < A.n; e += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t xb, yb, zb;
    double wph;
    m += photon_count(A, e, xb, yb, zb, wph);
  }
  for (int d = 32; d > 0; d >>= 1) m += __shfl_xor(m, d, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    if (m) atomicAdd(total, m);
  }
}

// Photons of the events: direction, distance, absorption point; the ones
// absorbed inside the box are appended to the particle arrays at *n_dev.
__global__ __launch_bounds__(256) void k_ph_emit(PhotoArgs A) {
#pragma clang fp contract(off)
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t e0 = wave * 64; e0 < A.n; e0 += waves * 64) {  // wave-uniform
    const uint64_t e = e0 + lane;
    uint32_t xb = 0, yb = 0, zb = 0, cnt = 0;
    double wph = 0.0;
    if (e < A.n) cnt = photon_count(A, e, xb, yb, zb, wph);
    uint32_t most = cnt;
    for (int d = 32; d > 0; d >>= 1) most = max(most, (uint32_t)__shfl_xor((int)most, d, 64));
    for (uint32_t j = 0; j < most; ++j) {
      bool keep = false;
      float px = 0.0f, py = 0.0f, pz = 0.0f;
      uint64_t id = 0;
      if (j < cnt) {
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
      if (m == 0) continue;
      unsigned long long base = 0;
      if (lane == (uint32_t)(__ffsll((unsigned long long)m) - 1)) base = atomicAdd(A.n_dev, (unsigned long long)__popcll(m));
      const int leader = __ffsll((unsigned long long)m) - 1;
      const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)base, leader);
      const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(base >> 32), leader);
      if (keep) {
        const uint64_t slot = (((uint64_t)hi << 32) | lo) + (uint64_t)__popcll(m & ((1ull << lane) - 1ull));
        A.x[slot] = px;
        A.y[slot] = py;
        A.z[slot] = pz;
        A.vx[slot] = 0.0f;
        A.vy[slot] = 0.0f;
        A.vz[slot] = 0.0f;
        A.w[slot] = (float)wph;
        A.id[slot] = id;
      }
    }
  }
}

static unsigned ph_blocks(uint64_t n) {
  const uint64_t b = (n + 255) / 256;
  return (unsigned)(b < 1024 ? (b > 0 ? b : 1) : 1024);
}

hipError_t launch_photo_count(const PhotoArgs& A, unsigned long long* total, hipStream_t s) {
  hipLaunchKernelGGL(k_ph_count, dim3(ph_blocks(A.n)), dim3(256), 0, s, A, total);
  return hipGetLastError();
}

hipError_t launch_photo_emit(const PhotoArgs& A, hipStream_t s) {
  hipLaunchKernelGGL(k_ph_emit, dim3(ph_blocks(A.n)), dim3(256), 0, s, A);
  return hipGetLastError();
}

}  // namespace pcmcc
