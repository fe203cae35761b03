// Device-side building blocks of one kinetic Monte-Carlo step (Tan, Carrey and
// Respaud, arXiv:1407.2737, Sec. II.1 steps iii-vii, Eqs. 2-5), all in FP64:
//   * Philox-4x64-10 counter-based uniforms (Salmon et al., SC'11);
//   * the Stoner-Wohlfarth stationary points of Eq. 2 in the particle's working plane;
//   * the "fall" into a basin, the two-state switching probability of Eq. 5 and the
//     jump draw, giving the particle's next moment.
//
// Stationary points are found from guaranteed brackets instead of a grid scan. With
// the field reflected into hx >= 0, hy >= 0 (theta -> pi - theta flips hx), the zeros
// of g(theta) = e'(theta)/2 = sin cos + hx sin - hy cos are: exactly one in
// (0, pi/2) (global minimum, g(0) = -hy < 0 < hx = g(pi/2)), exactly one in
// (pi, 3pi/2) (global maximum), none in (3pi/2, 2pi), and, strictly inside the
// astroid (hx^2 + hy^2 - 1)^3 + 27 hx^2 hy^2 < 0, a maximum and a metastable
// minimum in (pi/2, pi), on either side of the single zero t* of g' there
// (g'(pi/2) = hy - 1 < 0 < 1 - hx = g'(pi)). Each root is polished by Newton's
// method kept inside its bracket (bisection when a step leaves it).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mh {

constexpr double kPi = 3.14159265358979323846;
constexpr double kHalfPi = 1.57079632679489661923;

// ---------------------------------------------------------------------------
// Philox-4x64-10
// ---------------------------------------------------------------------------
constexpr uint64_t kPhM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2,
                                              uint64_t& c3, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kPhW0;
      k1 += kPhW1;
    }
    const uint64_t lo0 = kPhM0 * c0, hi0 = __umul64hi(kPhM0, c0);
    const uint64_t lo1 = kPhM1 * c2, hi1 = __umul64hi(kPhM1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

// Uniform in [0,1) for particle i at global step k: word (i mod 4) of the block at
// counter (i/4, k, 0, 0) under key (seed, stream), top 53 bits.
__device__ __forceinline__ double philox_uniform(uint64_t seed, uint64_t stream, int64_t i,
                                                 int64_t k) {
  uint64_t c0 = (uint64_t)(i >> 2), c1 = (uint64_t)k, c2 = 0, c3 = 0;
  philox4x64_10(c0, c1, c2, c3, seed, stream);
  const int w = (int)(i & 3);
  const uint64_t x = w == 0 ? c0 : (w == 1 ? c1 : (w == 2 ? c2 : c3));
  return (double)(x >> 11) * 0x1.0p-53;
}

// ---------------------------------------------------------------------------
// Stoner-Wohlfarth stationary points (reduced energy e = sin^2 - 2(hx cos + hy sin))
// ---------------------------------------------------------------------------
__device__ __forceinline__ double sw_energy(double s, double c, double hx, double hy) {
  return s * s - 2.0 * (hx * c + hy * s);
}

// g = e'/2 at t (returned) and dg/dt in gp.
__device__ __forceinline__ double sw_g(double t, double hx, double hy, double& gp) {
  double s, c;
  sincos(t, &s, &c);
  gp = (c * c - s * s) + hx * c + hy * s;
  return s * c + hx * s - hy * c;
}

// g' = e''/2 at t (returned) and its derivative in gpp.
__device__ __forceinline__ double sw_gp(double t, double hx, double hy, double& gpp) {
  double s, c;
  sincos(t, &s, &c);
  gpp = -4.0 * s * c - hx * s + hy * c;
  return (c * c - s * s) + hx * c + hy * s;
}

// Zero of f on (a, b) where f(a) < 0 iff a_neg; Newton kept inside the bracket.
template <bool kDeriv>
__device__ double bracketed_root(double a, double b, bool a_neg, double hx, double hy) {
  double x = 0.5 * (a + b);
  for (int it = 0; it < 200; ++it) {
    double d;
    const double f = kDeriv ? sw_gp(x, hx, hy, d) : sw_g(x, hx, hy, d);
    if (f == 0.0) return x;
    if ((f < 0.0) == a_neg)
      a = x;
    else
      b = x;
    double xn = x - f / d;
    if (!(xn > a && xn < b)) xn = 0.5 * (a + b);
    const double step = fabs(xn - x);
    x = xn;
    if (step <= 1e-15 * fmax(1.0, fabs(x)) || (b - a) <= 4e-16 * fmax(1.0, fabs(x))) break;
  }
  return x;
}

__device__ __forceinline__ double wrap_pi(double t) {
  // into (-pi, pi]
  if (t > kPi) t -= 2.0 * kPi;
  if (t <= -kPi) t += 2.0 * kPi;
  return t;
}

__device__ __forceinline__ bool astroid_bistable(double hx, double hy) {
  const double a = hx * hx + hy * hy - 1.0;
  return a * a * a + 27.0 * hx * hx * hy * hy < 0.0;
}

struct SWState {
  double th_c, e_c, th_o, e_o, e3;  // current/other minimum, lower maximum (units K V)
  bool two;
};

// Step iv-v: stationary points for (hx, hy) with hy >= 0, and the basin of theta0.
__device__ SWState sw_fall(double hx, double hy, double theta0) {
  SWState r;
  // ---- exact special cases (field along or across the axis) ----
  if (hy == 0.0) {
    const double e0 = -2.0 * hx, epi = 2.0 * hx;
    if (fabs(hx) < 1.0) {
      const double tm = acos(-hx);  // maxima at +-tm, both at energy 1 + hx^2
      const double at = fabs(theta0);
      bool to0;
      if (at < tm)
        to0 = true;
      else if (at > tm)
        to0 = false;
      else
        to0 = (e0 < epi) || (e0 == epi);  // tie on a maximum: lower energy, then nearer, then
                                          // the smaller angle (0)
      r.two = true;
      r.th_c = to0 ? 0.0 : kPi;
      r.e_c = to0 ? e0 : epi;
      r.th_o = to0 ? kPi : 0.0;
      r.e_o = to0 ? epi : e0;
      r.e3 = 1.0 + hx * hx;
    } else {
      r.two = false;
      r.th_c = r.th_o = hx > 0.0 ? 0.0 : kPi;
      r.e_c = r.e_o = hx > 0.0 ? e0 : epi;
      r.e3 = 0.0;
    }
    return r;
  }
  if (hx == 0.0) {
    if (hy < 1.0) {
      const double a = asin(hy);
      const double em = -hy * hy;  // both minima
      // basins: (-pi/2, pi/2) -> a ; (pi/2, 3pi/2) -> pi - a ; ties go to a
      const double t = theta0;
      const bool toa = (t > -kHalfPi && t < kHalfPi) || t == kHalfPi || t == -kHalfPi;
      r.two = true;
      r.th_c = toa ? a : kPi - a;
      r.th_o = toa ? kPi - a : a;
      r.e_c = r.e_o = em;
      r.e3 = 1.0 - 2.0 * hy;
    } else {
      r.two = false;
      r.th_c = r.th_o = kHalfPi;
      r.e_c = r.e_o = 1.0 - 2.0 * hy;
      r.e3 = 0.0;
    }
    return r;
  }
  // ---- general case: reflect into hx > 0 ----
  const bool refl = hx < 0.0;
  const double ax = fabs(hx);
  const double r1 = bracketed_root<false>(0.0, kHalfPi, true, ax, hy);        // global min
  const double r3 = bracketed_root<false>(kPi, 1.5 * kPi, false, ax, hy);     // global max
  double s, c;
  sincos(r1, &s, &c);
  const double e1 = sw_energy(s, c, ax, hy);
  bool two = false;
  double r2a = 0.0, r2b = 0.0, e2a = 0.0, e2b = 0.0;
  if (astroid_bistable(ax, hy)) {
    const double ts = bracketed_root<true>(kHalfPi, kPi, true, ax, hy);
    double d;
    if (sw_g(ts, ax, hy, d) < 0.0) {
      two = true;
      r2a = bracketed_root<false>(kHalfPi, ts, false, ax, hy);  // saddle maximum
      r2b = bracketed_root<false>(ts, kPi, true, ax, hy);       // metastable minimum
      sincos(r2a, &s, &c);
      e2a = sw_energy(s, c, ax, hy);
      sincos(r2b, &s, &c);
      e2b = sw_energy(s, c, ax, hy);
    }
  }
  const double back1 = refl ? wrap_pi(kPi - r1) : r1;
  if (!two) {
    r.two = false;
    r.th_c = r.th_o = back1;
    r.e_c = r.e_o = e1;
    r.e3 = 0.0;
    return r;
  }
  sincos(r3, &s, &c);
  const double e3g = sw_energy(s, c, ax, hy);
  const double e3 = fmin(e2a, e3g);
  // basin of theta0 in the reflected frame: the circle reads r1 (min) < r2a (max)
  // < r2b (min) < r3 (max) < r1 + 2 pi
  double x = refl ? (kPi - theta0) : theta0;
  // into [r3 - 2 pi, r3): theta0 lies in [-pi, pi], so one correction either way suffices
  if (x >= r3) x -= 2.0 * kPi;
  if (x < r3 - 2.0 * kPi) x += 2.0 * kPi;
  bool to1;
  if (x == r2a || x == r3 - 2.0 * kPi) {
    if (e1 != e2b) {
      to1 = e1 < e2b;
    } else {
      const double th1 = back1, th2 = refl ? wrap_pi(kPi - r2b) : wrap_pi(r2b);
      const double d1 = fabs(wrap_pi(theta0 - th1)), d2 = fabs(wrap_pi(theta0 - th2));
      to1 = (d1 < d2) || (d1 == d2 && th1 <= th2);
    }
  } else {
    to1 = x < r2a;
  }
  const double b1 = back1;
  const double b2 = refl ? wrap_pi(kPi - r2b) : wrap_pi(r2b);
  r.two = true;
  r.th_c = to1 ? b1 : b2;
  r.e_c = to1 ? e1 : e2b;
  r.th_o = to1 ? b2 : b1;
  r.e_o = to1 ? e2b : e1;
  r.e3 = e3;
  return r;
}

// ---------------------------------------------------------------------------
// Per-particle update (steps iii-vii)
// ---------------------------------------------------------------------------
struct NPParams {
  double BK_inv;    // 1 / (mu0 H_K) = Ms / (2 K), 1/T
  double BK;        // mu0 H_K, T (0 when K = 0)
  double beta;      // K V / (k_B T)
  double nu0dt;     // dt / tau0
  int prob_form;    // 0: Eq. 5, 1: single rate
  int thermal;      // T > 0
  int aniso;        // K > 0
};

struct NPResult {
  double mx, my, mz;
  double P;
  int jump;
  int two;
};

__device__ NPResult np_update(const NPParams& p, double Bx, double By, double Bz, double nx,
                              double ny, double nz, double mx, double my, double mz,
                              uint64_t seed, uint64_t stream, int64_t i, int64_t k) {
  NPResult out;
  out.P = 0.0;
  out.jump = 0;
  out.two = 0;
  if (!p.aniso) {  // K = 0: the moment aligns with the total field
    const double bn = sqrt(Bx * Bx + By * By + Bz * Bz);
    if (bn > 0.0) {
      out.mx = Bx / bn;
      out.my = By / bn;
      out.mz = Bz / bn;
    } else {
      out.mx = mx;
      out.my = my;
      out.mz = mz;
    }
    return out;
  }
  // step iii: working plane (n, u2)
  const double bpar = Bx * nx + By * ny + Bz * nz;
  double px = Bx - bpar * nx, py = By - bpar * ny, pz = Bz - bpar * nz;
  const double bp = sqrt(px * px + py * py + pz * pz);
  const double bn = sqrt(Bx * Bx + By * By + Bz * Bz);
  double ux, uy, uz, hy;
  if (bp > 1e-12 * fmax(bn, p.BK)) {
    ux = px / bp;
    uy = py / bp;
    uz = pz / bp;
    hy = bp * p.BK_inv;
  } else {
    hy = 0.0;
    const double mn = mx * nx + my * ny + mz * nz;
    double vx = mx - mn * nx, vy = my - mn * ny, vz = mz - mn * nz;
    const double vn = sqrt(vx * vx + vy * vy + vz * vz);
    if (vn > 1e-12) {
      ux = vx / vn;
      uy = vy / vn;
      uz = vz / vn;
    } else {
      // n x e, e = coordinate axis least aligned with n (first on ties)
      const double ax = fabs(nx), ay = fabs(ny), az = fabs(nz);
      int c = 0;
      if (ay < ax) c = 1;
      if (az < (c == 0 ? ax : ay)) c = 2;
      const double ex = c == 0, ey = c == 1, ez = c == 2;
      vx = ny * ez - nz * ey;
      vy = nz * ex - nx * ez;
      vz = nx * ey - ny * ex;
      const double wn = sqrt(vx * vx + vy * vy + vz * vz);
      ux = vx / wn;
      uy = vy / wn;
      uz = vz / wn;
    }
  }
  const double hx = bpar * p.BK_inv;
  const double theta0 = atan2(mx * ux + my * uy + mz * uz, mx * nx + my * ny + mz * nz);
  // steps iv-v
  const SWState sw = sw_fall(hx, hy, theta0);
  double th = sw.th_c;
  out.two = sw.two;
  // steps vi-vii
  if (p.thermal && sw.two) {
    const double a_c = p.beta * (sw.e3 - sw.e_c);
    const double a_o = p.beta * (sw.e3 - sw.e_o);
    double P;
    if (p.prob_form == 1) {
      P = -expm1(-p.nu0dt * exp(-a_c));
    } else {
      const double sig = 1.0 / (1.0 + exp(a_c - a_o));
      P = sig * (-expm1(-p.nu0dt * (exp(-a_c) + exp(-a_o))));
    }
    const double u = philox_uniform(seed, stream, i, k);
    out.P = P;
    if (u < P) {
      th = sw.th_o;
      out.jump = 1;
    }
  }
  double s, c;
  sincos(th, &s, &c);
  out.mx = c * nx + s * ux;
  out.my = c * ny + s * uy;
  out.mz = c * nz + s * uz;
  return out;
}

// Neumaier compensated accumulation: sum += x with running compensation.
__device__ __forceinline__ void neumaier_add(double& sum, double& comp, double x) {
  const double t = sum + x;
  if (fabs(sum) >= fabs(x))
    comp += (sum - t) + x;
  else
    comp += (x - t) + sum;
  sum = t;
}

}  // namespace mh
