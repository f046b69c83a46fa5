// The allocation-free charge deposit (pcmcc_deposit_noalloc): the same
// fixed-point CIC deposit as pcmcc_deposit, with the binned schedule's
// scratch (tile counts and starts, per-block tile tables, the tile-ordered
// particle copy, the range flag) carved out of one file-scope device array
// instead of library allocations, for callers that cannot allocate.
//
// Every GPU the library runs on holds its own copy of `scratch` (about
// 50 MiB) until the process ends.  Host code never passes the array's name to
// a kernel or a copy: there the name is a host-side stand-in, not a device
// address.  The device address of each GPU's copy is looked up once, at
// context creation with that device current (noalloc_setup), and kept per
// device; only that address is used.  All calls on one GPU share its copy, so
// calls that overlap on one GPU race.
#include <mutex>

#include "pcmcc_runtime.hpp"

namespace {

// Largest inputs of the allocation-free deposit.
constexpr uint64_t kNoallocMaxParticles = 1ull << 21;  // particles per call
constexpr uint64_t kNoallocMaxTiles = 1ull << 18;      // 8^3-cell tiles (a 512^3 grid)

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
// Layout: range flag | tile counts | tile starts | per-block tile tables |
// tile-ordered particles.
constexpr size_t kOffFlag = 0;
constexpr size_t kOffCount = 256;
constexpr size_t kOffStart = kOffCount + align256((kNoallocMaxTiles + 1) * sizeof(uint32_t));
constexpr size_t kOffDump = kOffStart + align256((kNoallocMaxTiles + 1) * sizeof(uint32_t));
constexpr size_t kOffSorted = kOffDump + align256(kNoallocMaxParticles * sizeof(uint2));
constexpr size_t kScratchBytes = kOffSorted + align256(kNoallocMaxParticles * sizeof(float4));

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_looked_up[kMaxDevices] = {};
unsigned char* g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};

}  // namespace

namespace pcmcc_rt {

// Looks up the device address of this device's scratch array, once per
// device; the device must be current.
void noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_looked_up[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_err[device] = e;
  g_ptr[device] = e == hipSuccess ? static_cast<unsigned char*>(p) : nullptr;
  if (e != hipSuccess) (void)hipGetLastError();
  g_looked_up[device] = true;
}

}  // namespace pcmcc_rt

extern "C" {

int pcmcc_deposit_noalloc(pcmcc_ctx* c, const float* x, const float* y, const float* z, const float* w,
                          const int64_t* n_dev, const pcmcc_grid* grid, int64_t* rho) {
  if (!c) return fail(nullptr, PCMCC_EINVAL, "null context");
  if (!x || !y || !z || !w || !n_dev || !rho) return fail(c, PCMCC_EINVAL, "null array");
  if (!grid || grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || !(grid->dx > 0))
    return fail(c, PCMCC_EINVAL, "invalid grid");
  const int dev = c->device;
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (dev < 0 || dev >= kMaxDevices || !g_looked_up[dev])
      return fail(c, PCMCC_ESTATE, "allocation-free scratch of device %d was not set up", dev);
    if (!g_ptr[dev])
      return fail(c, PCMCC_EHIP, "allocation-free scratch of device %d unavailable: %s", dev,
                  hipGetErrorString(g_err[dev]));
    base = g_ptr[dev];
  }
  HIP_TRY(c, hipSetDevice(dev));
  HIP_TRY(c, hipMemcpyAsync(c->host_n, n_dev, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int64_t n = *c->host_n;
  if (n < 0) return fail(c, PCMCC_EINVAL, "negative particle count");
  unsigned* flag = reinterpret_cast<unsigned*>(base + kOffFlag);
  const DepositGeom g{grid->nx, grid->ny, grid->nz, grid->x0, grid->y0, grid->z0, 1.0 / grid->dx, flag};
  const DepositNeeds d = deposit_needs(g, (uint64_t)n);
  if ((uint64_t)n > kNoallocMaxParticles)
    return fail(c, PCMCC_EINVAL, "%lld particles exceed the allocation-free deposit's maximum of %llu",
                (long long)n, (unsigned long long)kNoallocMaxParticles);
  if (d.n_tiles > kNoallocMaxTiles)
    return fail(c, PCMCC_EINVAL, "%llu tiles of 8^3 cells exceed the allocation-free deposit's maximum of %llu",
                (unsigned long long)d.n_tiles, (unsigned long long)kNoallocMaxTiles);
  if (d.dump_entries > kNoallocMaxParticles || d.sorted > kNoallocMaxParticles)
    return fail(c, PCMCC_EINVAL, "deposit work exceeds the allocation-free scratch");
  HIP_TRY(c, launch_fill_u32(flag, 1, 0u, c->stream));
  if (!d.binned) {
    HIP_TRY(c, launch_deposit(x, y, z, w, n_dev, g, rho, c->stream));
  } else {
    DepositWork W;
    W.tile_count = reinterpret_cast<uint32_t*>(base + kOffCount);
    W.tile_start = reinterpret_cast<uint32_t*>(base + kOffStart);
    W.dump = reinterpret_cast<uint2*>(base + kOffDump);
    W.sorted = reinterpret_cast<float4*>(base + kOffSorted);
    HIP_TRY(c, launch_deposit_binned(x, y, z, w, (uint64_t)n, g, rho, W, c->stream));
  }
  HIP_TRY(c, hipMemcpyAsync(c->host_err, flag, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (*c->host_err)
    return fail(c, PCMCC_ERANGE, "charge outside the deposit's fixed-point range (a weight outside [0, 2^31) or "
                "more than 2^31 electrons in one cell)");
  return PCMCC_OK;
}

}  // extern "C"
