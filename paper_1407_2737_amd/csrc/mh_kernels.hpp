// Shared host/device descriptors of the kMC step kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mh_device.hpp"

namespace mh {

struct alignas(32) D4 {
  double x, y, z, w;
};
struct alignas(16) F4 {
  float x, y, z, w;
};

// Everything one (assembly, replica) system needs on the device.
struct SysDesc {
  const D4* pos64;   // positions / d (reduced units), n entries
  const F4* pos32;   // same in FP32
  const D4* axes;    // easy axes (unit), n entries (this replica's axis set)
  D4* m64;           // FP64 moments, buffer b at m64 + b * stride
  F4* m32;           // FP32 copy used by FP32 field sums, same layout
  double* area;      // per-particle area accumulators: [n] sums then [n] compensations
  double* recpart;   // loop record partial sums [n_kept * S][ntiles]
  double* diag;      // optional per-particle diagnostics (8 doubles each) or null
  D4* field;         // reduced dipolar sum per particle, written by the field kernel
  double* rec;       // loop record of the kept steps: sum_i m_x after each step
  double* sys_area;  // this system's loop area (J/m^3), written at the end of a run
  int64_t stride;    // distance between the two moment buffers (elements)
  uint64_t seed, stream;
  NPParams np;
  double Bmax;       // mu0 Hmax (T)
  double Bscale;     // mu0 Ms / 24: field unit of the reduced dipolar sum (T)
  double Ms;
  int32_t n;
  int32_t ntiles;    // update blocks of 256 particles (1 for the resident kernel)
  int32_t S, total_steps, kept0, static_field;
  int32_t field_only;  // diagnostics: write the dipolar field to diag, change nothing
  int32_t pad_;
};

__host__ __device__ inline double applied_field(const SysDesc& s, int64_t k) {
  if (s.static_field) return s.Bmax;
  return s.Bmax * cos(2.0 * kPi * (double)k / (double)s.S);
}

}  // namespace mh
