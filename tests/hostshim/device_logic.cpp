// Host build of the device-side step logic (Philox, Stoner-Wohlfarth extrema and fall,
// per-particle update) so that the CPU test suite can compare it with the oracle.
// Test infrastructure only: the GPU library is built from the same header by hipcc.
#include <cmath>
#include <cstdint>
#include <vector>
#define __device__
#define __host__
#define __forceinline__ inline
#define __noinline__ __attribute__((noinline))
#define HIP_INCLUDE_HIP_HIP_RUNTIME_H
static inline uint64_t __umul64hi(uint64_t a, uint64_t b) {
  return (uint64_t)(((__uint128_t)a * b) >> 64);
}
static inline void host_sincosf(float t, float* s, float* c) {
  *s = std::sin(t);
  *c = std::cos(t);
}
#define __sincosf host_sincosf
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_rsq(x) (1.0 / std::sqrt(x))
using std::fabs;
using std::fmax;
using std::copysign;
using std::isnan;
using std::remainder;
using std::fmin;
#include "../../paper_1407_2737_amd/csrc/mh_device.hpp"

extern "C" {

void dl_philox(uint64_t seed, uint64_t stream, int64_t nblk, const uint64_t* ctr, uint64_t* out) {
  for (int64_t b = 0; b < nblk; ++b) {
    uint64_t c0 = ctr[4 * b], c1 = ctr[4 * b + 1], c2 = ctr[4 * b + 2], c3 = ctr[4 * b + 3];
    mh::philox4x64_10(c0, c1, c2, c3, seed, stream);
    out[4 * b] = c0;
    out[4 * b + 1] = c1;
    out[4 * b + 2] = c2;
    out[4 * b + 3] = c3;
  }
}

void dl_sw(int64_t n, const double* hx, const double* hy, const double* th0, double* out) {
  for (int64_t i = 0; i < n; ++i) {
    const mh::Dir d = {std::sin(th0[i]), std::cos(th0[i])};
    const mh::SWState r = mh::sw_fall(hx[i], hy[i], d);
    double* o = out + 6 * i;
    o[0] = std::atan2(r.s_c, r.c_c);
    o[1] = r.e_c;
    o[2] = std::atan2(r.s_o, r.c_o);
    o[3] = r.e_o;
    o[4] = r.e3;
    o[5] = r.two ? 1.0 : 0.0;
  }
}

// As dl_sw with step iv as the 200-point scan.
void dl_sw_scan200(int64_t n, const double* hx, const double* hy, const double* th0,
                   double* out) {
  for (int64_t i = 0; i < n; ++i) {
    const mh::Dir d = {std::sin(th0[i]), std::cos(th0[i])};
    const mh::SWState r = mh::sw_fall_scan200(hx[i], hy[i], d);
    double* o = out + 6 * i;
    o[0] = std::atan2(r.s_c, r.c_c);
    o[1] = r.e_c;
    o[2] = std::atan2(r.s_o, r.c_o);
    o[3] = r.e_o;
    o[4] = r.e3;
    o[5] = r.two ? 1.0 : 0.0;
  }
}

// B, n, m: n x 3; out: n x 6 (new moment, P, jump, two)
void dl_update(int64_t n, const double* B, const double* ax, const double* m, double BK,
               double beta, double nu0dt, int prob_form, int thermal, uint64_t seed,
               uint64_t stream, int64_t k, int scan200, double* out) {
  mh::NPParams p;
  p.BK = BK;
  p.BK_inv = 1.0 / BK;
  p.beta = beta;
  p.nu0dt = nu0dt;
  p.prob_form = prob_form;
  p.thermal = thermal;
  p.aniso = 1;
  p.scan200 = scan200;
  for (int64_t i = 0; i < n; ++i) {
    const mh::NPResult r =
        mh::np_update<true>(p, B[3 * i], B[3 * i + 1], B[3 * i + 2], ax[3 * i], ax[3 * i + 1],
                      ax[3 * i + 2], m[3 * i], m[3 * i + 1], m[3 * i + 2], seed, stream, i, k);
    double* o = out + 6 * i;
    o[0] = r.mx;
    o[1] = r.my;
    o[2] = r.mz;
    o[3] = r.P;
    o[4] = r.jump;
    o[5] = r.two;
  }
}

// Mean-magnetisation loop of n non-interacting particles, as the GPU kernel runs it:
// per step every particle's master_step, then the loop record (M_S <m . e_H> for each
// kept step, n_kept x S) and the per-particle compensated area averaged over particles
// and kept periods (area_out[0], J/m^3). eh: unit field direction.
void dl_master(int64_t n, const double* ax, double Ms, double BK, double beta, double nu0dt,
               int prob_form, int thermal, double Bmax, int S, int n_periods, int n_discard,
               int static_field, const double* eh, double* M_out, double* area_out) {
  mh::NPParams p;
  p.BK = BK;
  p.BK_inv = 1.0 / BK;
  p.beta = beta;
  p.nu0dt = nu0dt;
  p.prob_form = prob_form;
  p.thermal = thermal;
  p.aniso = 1;
  p.scan200 = 0;
  std::vector<mh::MasterState> q((size_t)n);
  std::vector<double> prev((size_t)n), sum((size_t)n, 0.0), comp((size_t)n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    mh::master_init(q[i], ax[3 * i], ax[3 * i + 1], ax[3 * i + 2], eh[0], eh[1], eh[2]);
    prev[i] = q[i].ax * eh[0] + q[i].ay * eh[1] + q[i].az * eh[2];
  }
  const int total = S * n_periods, kept0 = S * n_discard;
  for (int k = 0; k < total; ++k) {
    const double Bext = static_field ? Bmax : Bmax * std::cos(2.0 * mh::kPi * (double)k / (double)S);
    double msum = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double mx = mh::master_step(p, Bext, eh[0], eh[1], eh[2], ax[3 * i], ax[3 * i + 1],
                                        ax[3 * i + 2], q[i]);
      if (k >= kept0) mh::neumaier_add(sum[i], comp[i], Ms * Bext * (mx - prev[i]));
      prev[i] = mx;
      msum += mx;
    }
    if (k >= kept0) M_out[k - kept0] = Ms * msum / (double)n;
  }
  double a = 0.0;
  for (int64_t i = 0; i < n; ++i) a += sum[i] + comp[i];
  area_out[0] = a / ((double)n * (n_periods - n_discard));
}

// The 128-bit products of the two Philox multipliers (lo, hi words per input).
void dl_mul128(int64_t n, const uint64_t* x, uint64_t* out) {
  for (int64_t q = 0; q < n; ++q) {
    mh::mul128<mh::kPhM0>(x[q], out[4 * q], out[4 * q + 1]);
    mh::mul128<mh::kPhM1>(x[q], out[4 * q + 2], out[4 * q + 3]);
  }
}
}
