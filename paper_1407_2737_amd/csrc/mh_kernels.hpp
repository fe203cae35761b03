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

// Loop record partial sums per 256-particle update block. A system that may run under
// k_update3 (R x ntiles <= kUpdate3MaxBlocks update blocks, the launches of at most that
// many use it) keeps one per 64-lane wave, as k_update3 runs each block as four
// sub-blocks: a row's value is then the sum over blocks, in block order, of
// (w0 + w1) + (w2 + w3), and a kernel that forms a block's total itself stores it in
// slot 0 and zeros in the others. Larger systems keep the block total alone (rec_slots
// = 1), the same value.
constexpr int kRecSlots = 4;
constexpr int kUpdate3MaxBlocks = 256;
inline int rec_slots_for(int64_t R, int64_t ntiles) {
  return R * ntiles <= kUpdate3MaxBlocks ? kRecSlots : 1;
}

// Everything one (assembly, replica) system needs on the device.
struct SysDesc {
  const D4* pos64;   // positions / d (reduced units), n entries
  const F4* pos32;   // same in FP32
  const D4* axes;    // easy axes (unit), n entries (this replica's axis set)
  D4* m64;           // FP64 moments, buffer b at m64 + b * stride
  F4* m32;           // FP32 copy used by FP32 field sums, same layout
  double* area;      // per-particle area accumulators: [n] sums then [n] compensations
  double* recpart;   // loop record partial sums [n_kept * S][ntiles][rec_slots]
  double* diag;      // optional per-particle diagnostics (8 doubles each) or null
  D4* field;         // reduced dipolar sums, nsplit partial sums per particle ([part][n])
  F4* field32;       // the same partial sums in FP32 (FP32 field form; field is then null)
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
  int32_t rec_slots;   // loop record partial sums per update block (1 or kRecSlots)
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

// One system's share of a launch that covers several matrix-form systems: its
// operands and its range of blocks (product: row tiles x replica tiles x k splits; update:
// nbx particle blocks of 256 x R replicas, its replica 0 at index `first` of the launch's
// descriptor array).
struct WMGroupItem {
  WMArgs g;
  int32_t boff;   // first block of the item in the launch
  int32_t nb;     // blocks of the item
  int32_t first;  // update: descriptor index of replica 0
  int32_t nbx;    // update: particle blocks per replica
};

// Reads the descriptor fields that a kernel's step-window test and first data loads
// depend on, all ahead of any branch, and holds them together in scalar registers: the
// scalar loads are then issued back to back and share one wait, where the compiler would
// otherwise place each behind the branch that first needs it (one round trip each).
// Later reads of these fields reuse the values (the descriptors are not written by the
// kernels that read them).
// The step base of a launch: *kbase (a captured graph's device-side counter), or 0
// without one. The load itself is unconditional (from `fallback`, any readable address,
// when kbase is null), so it is issued with the launch's first scalar loads rather than
// behind a branch.
__device__ __forceinline__ int64_t step_base(const int64_t* kbase, const void* fallback) {
  const int64_t v = *(kbase ? kbase : reinterpret_cast<const int64_t*>(fallback));
  return kbase ? v : 0;
}

__device__ __forceinline__ void desc_prefetch(const SysDesc& s, const void* e0 = nullptr,
                                              const void* e1 = nullptr, const void* e2 = nullptr,
                                              const void* e3 = nullptr, const void* e4 = nullptr,
                                              double e5 = 0.0) {
  // e0..e5: further uniform values the caller read from descriptors, held in the same
  // batch
  const int64_t ko = s.k_origin, sd = s.stride;
  const int32_t n = s.n, ts = s.total_steps, np = s.nsplit, fo = s.field_only;
  const void* q0 = s.m64;
  const void* q1 = s.axes;
  const void* q2 = s.field32;
  const void* q3 = s.field;
  asm volatile("" ::"s"(ko), "s"(sd), "s"(n), "s"(ts), "s"(np), "s"(fo), "s"(q0), "s"(q1), "s"(q2),
               "s"(q3), "s"(e0), "s"(e1), "s"(e2), "s"(e3), "s"(e4), "s"(e5));
}

__host__ __device__ inline double applied_field(const SysDesc& s, int64_t k) {
  if (s.static_field) return s.Bmax;
  return s.Bmax * cos(2.0 * kPi * (double)k / (double)s.S);
}

// v of the lane N places along in the lane's row of 16 (DPP row rotation).
template <int N>
__device__ __forceinline__ double dpp_row_ror(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, 0x120 + N, 0xF, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), 0x120 + N, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over a wave's 64 lanes (all active), every lane getting the total, in a fixed
// tree: lane l adds lane l ^ 32, then l ^ 16, ..., l ^ 1. The last four steps are DPP
// rotations within rows of 16, which fetch lane l ^ 8, ^ 4, ^ 2, ^ 1 once the values
// repeat with period 16, 8, 4 and 2 along the row (as they do after the steps before),
// at register latency instead of an LDS permute's.
__device__ __forceinline__ double wave_sum(double v) {
  v += __shfl_xor(v, 32, 64);
  v += __shfl_xor(v, 16, 64);
  v += dpp_row_ror<8>(v);
  v += dpp_row_ror<4>(v);
  v += dpp_row_ror<2>(v);
  v += dpp_row_ror<1>(v);
  return v;
}

// Loads through the global address space as one vector. The pointers come from
// descriptors in memory, where the compiler cannot infer the address space and would
// emit flat loads, whose waits also wait on LDS and scalar loads.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ F4 ldg(const F4* p) {
  const f4v v = *(const __attribute__((address_space(1))) f4v*)p;
  return F4{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ D4 ldg(const D4* p) {
  const d4v v = *(const __attribute__((address_space(1))) d4v*)p;
  return D4{v.x, v.y, v.z, v.w};
}

// Inputs of steps iii-vii for particle i of system s from the reduced dipolar sum
// (ax, ay, az) and the moments of buffer cur: the applied and total field, the moment
// and the axis.
struct NPIn {
  double Bext, Bx, By, Bz;
  D4 mo, nn;
};

__device__ __forceinline__ NPIn np_in(const SysDesc& s, int64_t k, double ax, double ay,
                                      double az, const D4& mo, const D4& nn) {
  NPIn q;
  q.Bext = applied_field(s, k);
  const double ex = s.eh[0], ey = s.eh[1], ez = s.eh[2];
  q.Bx = s.Bscale * ax + q.Bext * ex;
  q.By = s.Bscale * ay + q.Bext * ey;
  q.Bz = s.Bscale * az + q.Bext * ez;
  q.mo = mo;
  q.nn = nn;
  return q;
}

__device__ __forceinline__ NPIn np_in(const SysDesc& s, int i, int64_t k, int cur, double ax,
                                      double ay, double az) {
  return np_in(s, k, ax, ay, az, s.m64[(int64_t)cur * s.stride + i], s.axes[i]);
}

// Sum of the nsplit partial fields of particle i in part order, in FP64 (the parts are
// FP64, or FP32 for the FP32 field form). The loads of four parts at a time are issued
// together (addresses of missing parts fall back to part 0 and their terms are skipped),
// so a few parts cost one memory round trip, not one each.
template <typename P4>
__device__ __forceinline__ void sum_parts_of(const P4* field, int nsplit, int64_t n, int i,
                                             double& fx, double& fy, double& fz) {
  fx = fy = fz = 0.0;
  for (int p0 = 0; p0 < nsplit; p0 += 4) {
    const P4* b = field + (int64_t)p0 * n + i;
    const int m = nsplit - p0;
    const P4 f0 = ldg(b);
    const P4 f1 = ldg(b + (m > 1 ? n : 0));
    const P4 f2 = ldg(b + (m > 2 ? 2 * n : 0));
    const P4 f3 = ldg(b + (m > 3 ? 3 * n : 0));
    fx += (double)f0.x;
    fy += (double)f0.y;
    fz += (double)f0.z;
    fx = m > 1 ? fx + (double)f1.x : fx;
    fy = m > 1 ? fy + (double)f1.y : fy;
    fz = m > 1 ? fz + (double)f1.z : fz;
    fx = m > 2 ? fx + (double)f2.x : fx;
    fy = m > 2 ? fy + (double)f2.y : fy;
    fz = m > 2 ? fz + (double)f2.z : fz;
    fx = m > 3 ? fx + (double)f3.x : fx;
    fy = m > 3 ? fy + (double)f3.y : fy;
    fz = m > 3 ? fz + (double)f3.z : fz;
  }
}

__device__ __forceinline__ void sum_parts(const SysDesc& s, int i, double& fx, double& fy,
                                          double& fz) {
  if (s.field32)
    sum_parts_of(s.field32, s.nsplit, s.n, i, fx, fy, fz);
  else
    sum_parts_of(s.field, s.nsplit, s.n, i, fx, fy, fz);
}

// Eq. 6: the dipolar field along e_H in the +Hmax step (k = 0 mod S) minus that in the
// -Hmax step (k = S/2 mod S), over the kept periods.
__device__ __forceinline__ void np_dhdip(const SysDesc& s, int i, int64_t k, double ax, double ay,
                                         double az) {
  if (s.dhdip && k >= s.kept0) {
    const int64_t ph = k % s.S;
    const double ex = s.eh[0], ey = s.eh[1], ez = s.eh[2];
    const double bh = s.Bscale * ax * ex + s.Bscale * ay * ey + s.Bscale * az * ez;
    if (ph == 0)
      s.dhdip[i] += bh;
    else if (ph == s.S / 2)
      s.dhdip[i] -= bh;
  }
}

// Outputs of the step: the new moment into buffer cur^1 (and its FP32 copy, and *mnew
// when given), the area, the diagnostics; returns the new moment's component along e_H.
// acc, when given, holds the particle's area accumulator (sum, compensation) in the
// caller's registers: it is read from there instead of memory and kept up to date (the
// memory copy is written as well).
__device__ __forceinline__ double np_out(const SysDesc& s, int i, int64_t k, int cur,
                                         const NPIn& q, const NPResult& r, double* acc = nullptr,
                                         D4* mnew = nullptr) {
  const double ex = s.eh[0], ey = s.eh[1], ez = s.eh[2];
  const int nxt = cur ^ 1;
  D4 mn;
  mn.x = r.mx;
  mn.y = r.my;
  mn.z = r.mz;
  mn.w = 0.0;
  s.m64[(int64_t)nxt * s.stride + i] = mn;
  if (mnew) *mnew = mn;
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
    const D4& mo = q.mo;
    const double mh_old = mo.x * ex + mo.y * ey + mo.z * ez;
    double sum = acc ? acc[0] : s.area[i], comp = acc ? acc[1] : s.area[s.n + i];
    neumaier_add(sum, comp, s.Ms * q.Bext * (mh_new - mh_old));
    s.area[i] = sum;
    s.area[s.n + i] = comp;
    if (acc) {
      acc[0] = sum;
      acc[1] = comp;
    }
  }
  if (s.diag) {
    double* d = s.diag + (int64_t)i * 8;
    d[0] = q.Bx;
    d[1] = q.By;
    d[2] = q.Bz;
    d[3] = r.P;
    d[4] = (double)r.jump;
    d[5] = (double)r.two;
    d[6] = 0.0;
    d[7] = 0.0;
  }
  return mh_new;
}

// The moment of particle i in buffer cur and its axis: loaded before the field sums
// are added, so that these loads and the partial-sum loads make one memory round trip.
struct NPState {
  D4 mo, nn;
};
__device__ __forceinline__ NPState np_state(const SysDesc& s, int i, int cur) {
  return NPState{ldg(s.m64 + (int64_t)cur * s.stride + i), ldg(s.axes + i)};
}

// Steps iii-vii for particle i of system s with the reduced dipolar sum (ax, ay, az)
// from the moment and axis st (buffer cur); writes buffer cur^1, accumulates the area,
// and returns the new moment's component along the field direction e_H. kScan as for
// np_update; acc and mnew as for np_out.
template <bool kScan>
__device__ __forceinline__ double np_epilogue(const SysDesc& s, int i, int64_t k, int cur,
                                              double ax, double ay, double az,
                                              const NPState& st, double* acc = nullptr,
                                              D4* mnew = nullptr) {
  if (s.field_only) {
    double* d = s.diag + (int64_t)i * 8;
    d[0] = s.Bscale * ax;
    d[1] = s.Bscale * ay;
    d[2] = s.Bscale * az;
    return 0.0;
  }
  np_dhdip(s, i, k, ax, ay, az);
  const NPIn q = np_in(s, k, ax, ay, az, st.mo, st.nn);
  const NPResult r = np_update<kScan>(s.np, q.Bx, q.By, q.Bz, q.nn.x, q.nn.y, q.nn.z, q.mo.x,
                                      q.mo.y, q.mo.z, s.seed, s.stream, i, k);
  return np_out(s, i, k, cur, q, r, acc, mnew);
}

template <bool kScan>
__device__ __forceinline__ double np_epilogue(const SysDesc& s, int i, int64_t k, int cur,
                                              double ax, double ay, double az) {
  return np_epilogue<kScan>(s, i, k, cur, ax, ay, az, np_state(s, i, cur));
}

}  // namespace mh
