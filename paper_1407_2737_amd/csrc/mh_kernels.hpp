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
  D4* field;         // reduced dipolar sums, nsplit partial sums per particle ([part][n])
  double* rec;       // loop record of the kept steps: sum_i m_x after each step
  double* sys_area;  // this system's loop area (J/m^3), written at the end of a run
  double* dhdip;     // per-particle Eq. 6 sums over kept periods (T), or null
  int64_t stride;    // distance between the two moment buffers (elements)
  int64_t k_origin;  // global step at which this system's step 0 runs
  uint64_t seed, stream;
  NPParams np;
  double Bmax;       // mu0 Hmax (T)
  double Bscale;     // mu0 Ms / 24: field unit of the reduced dipolar sum (T)
  double eh[3];      // unit direction of the applied field
  double Ms;
  int32_t n;
  int32_t ntiles;    // update blocks of 256 particles (1 for the resident kernel)
  int32_t S, total_steps, kept0, static_field;
  int32_t field_only;  // diagnostics: write the dipolar field to diag, change nothing
  int32_t nsplit;      // source parts of the tiled field sum (partials summed by the update)
};

// Operands of the interaction-matrix product (see mh_wm.hip).
struct WMArgs {
  const D4* pos;   // positions in units of d (the W tiles are generated from them)
  int n;           // particles
  __bf16* mhi;     // M^T hi: Rp x Kp, fragment-major (see mt_offset in mh_wm.hip)
  __bf16* mlo;     // M^T lo
  float* bt;       // B^T: Rp x Mp (reduced dipolar sums)
  int Mp, Kp, Rp;
  int n_rtiles;    // Mp / WM_BN
  int n_ctiles;    // Rp / WM_BM
};

__host__ __device__ inline double applied_field(const SysDesc& s, int64_t k) {
  if (s.static_field) return s.Bmax;
  return s.Bmax * cos(2.0 * kPi * (double)k / (double)s.S);
}

// Steps iii-vii for particle i of system s with the reduced dipolar sum (ax, ay, az)
// from the moments in buffer cur; writes buffer cur^1, accumulates the area, and
// returns the new moment's component along the field direction e_H. kScan as for
// np_update.
template <bool kScan>
__device__ inline double np_epilogue(const SysDesc& s, int i, int64_t k, int cur, double ax, double ay,
                              double az) {
  if (s.field_only) {
    double* d = s.diag + (int64_t)i * 8;
    d[0] = s.Bscale * ax;
    d[1] = s.Bscale * ay;
    d[2] = s.Bscale * az;
    return 0.0;
  }
  const double Bext = applied_field(s, k);
  const double ex = s.eh[0], ey = s.eh[1], ez = s.eh[2];
  const double Bx = s.Bscale * ax + Bext * ex, By = s.Bscale * ay + Bext * ey,
               Bz = s.Bscale * az + Bext * ez;
  if (s.dhdip && k >= s.kept0) {
    // Eq. 6: the dipolar field along e_H in the +Hmax step (k = 0 mod S) minus that in
    // the -Hmax step (k = S/2 mod S)
    const int64_t ph = k % s.S;
    const double bh = s.Bscale * ax * ex + s.Bscale * ay * ey + s.Bscale * az * ez;
    if (ph == 0)
      s.dhdip[i] += bh;
    else if (ph == s.S / 2)
      s.dhdip[i] -= bh;
  }
  const D4 mo = s.m64[(int64_t)cur * s.stride + i];
  const D4 nn = s.axes[i];
  const NPResult r =
      np_update<kScan>(s.np, Bx, By, Bz, nn.x, nn.y, nn.z, mo.x, mo.y, mo.z, s.seed, s.stream, i, k);
  const int nxt = cur ^ 1;
  D4 mn;
  mn.x = r.mx;
  mn.y = r.my;
  mn.z = r.mz;
  mn.w = 0.0;
  s.m64[(int64_t)nxt * s.stride + i] = mn;
  if (s.m32) {
    F4 mf;
    mf.x = (float)r.mx;
    mf.y = (float)r.my;
    mf.z = (float)r.mz;
    mf.w = 0.f;
    s.m32[(int64_t)nxt * s.stride + i] = mf;
  }
  const double mh_new = r.mx * ex + r.my * ey + r.mz * ez;
  if (k >= s.kept0) {
    const double mh_old = mo.x * ex + mo.y * ey + mo.z * ez;
    double sum = s.area[i], comp = s.area[s.n + i];
    neumaier_add(sum, comp, s.Ms * Bext * (mh_new - mh_old));
    s.area[i] = sum;
    s.area[s.n + i] = comp;
  }
  if (s.diag) {
    double* d = s.diag + (int64_t)i * 8;
    d[0] = Bx;
    d[1] = By;
    d[2] = Bz;
    d[3] = r.P;
    d[4] = (double)r.jump;
    d[5] = (double)r.two;
    d[6] = 0.0;
    d[7] = 0.0;
  }
  return mh_new;
}

}  // namespace mh
