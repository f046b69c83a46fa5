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
  // output: particle arrays, appended at *n_dev
  float *x, *y, *z, *vx, *vy, *vz, *w;
  uint64_t* id;
  unsigned long long* n_dev;
};

hipError_t launch_photo_count(const PhotoArgs& A, unsigned long long* total, hipStream_t s);
hipError_t launch_photo_emit(const PhotoArgs& A, hipStream_t s);

}  // namespace pcmcc
