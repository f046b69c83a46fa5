// Device-side declarations of the discrete photoionization.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pcmcc_device.hpp"

namespace pcmcc {

struct PhotoArgs {
  const float *ex, *ey, *ez, *ew;  // ionization events
  uint64_t n;
  double eta, w_ph;     // photons per ionization, photon weight (<= 0: the event's)
  double k1, k2, ln_k;  // absorption coefficients, ln(k2 / k1)
  double s_lo, s_hi;    // bisection range of ln r
  Key key;
  double lo[3], hi[3];  // grid box
  const uint64_t* offs;  // exclusive scan of the photon counts (emission)
  uint64_t total;        // photons (emission)
  // output: particle arrays, appended at *n_dev
  float *x, *y, *z, *vx, *vy, *vz, *w;
  uint64_t* id;
  unsigned long long* n_dev;
};

// Temporary bytes of the scan of n counts.
hipError_t photo_scan_bytes(uint64_t n, size_t* bytes);
// counts[e] of the A.n events and their exclusive scan offs[e].
hipError_t launch_photo_count(const PhotoArgs& A, uint32_t* counts, void* temp, size_t temp_bytes, uint64_t* offs,
                              hipStream_t s);
// The A.total photons (A.offs set), appended at A.n_dev.
hipError_t launch_photo_emit(const PhotoArgs& A, hipStream_t s);

}  // namespace pcmcc
