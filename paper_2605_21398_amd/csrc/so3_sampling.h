// Orientation samplers on the device (Sec. IV-C): the Super-Fibonacci
// sequence for the global search and GeoBall-SF for the local search in a
// geodesic ball.  Unit quaternions, scalar first, float32.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace regdock {

// Points of the tabulated radial distribution function of GeoBall-SF.
constexpr int GEOBALL_TABLE = 4096;

hipError_t super_fibonacci(int n, float* out, hipStream_t s);

// q0 need not be unit (it is normalised); theta in (0, pi/2]; gamma <= 0 means
// gamma = n.  Blocks until the samples are written (the radial table is
// built on the host and released after the kernel).
hipError_t geoball_sf(int n, const double* q0, double theta, double gamma, float* out, hipStream_t s);

// The same samples with the radial table built on the device in a static
// device array (no allocation, no host copy); asynchronous on s.  Calls that
// overlap on one device share the table and race.
hipError_t geoball_sf_noalloc(int n, const double* q0, double theta, double gamma, float* out, hipStream_t s);

}  // namespace regdock
