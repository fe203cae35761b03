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

// FP32 seed of a zero of g (kDeriv = false) or of g' (kDeriv = true) on (a, b), where the
// function is negative at a iff a_neg: Newton kept inside the bracket, bisection when a
// step leaves it. Accurate to the single-precision sine/cosine (about 1e-6).
template <bool kDeriv>
__device__ float seed_root(float a, float b, bool a_neg, float hx, float hy) {
  float x = 0.5f * (a + b);
  for (int it = 0; it < 30; ++it) {
    float s, c;
    __sincosf(x, &s, &c);
    float f, d;
    if (kDeriv) {
      f = (c * c - s * s) + hx * c + hy * s;
      d = -4.f * s * c - hx * s + hy * c;
    } else {
      f = s * c + hx * s - hy * c;
      d = (c * c - s * s) + hx * c + hy * s;
    }
    if ((f < 0.f) == a_neg)
      a = x;
    else
      b = x;
    const float dx = -f / d;
    if (fabsf(dx) < 1e-6f) break;  // converged to single precision
    float xn = x + dx;
    if (!(xn > a && xn < b)) xn = 0.5f * (a + b);
    x = xn;
  }
  return x;
}

// FP64 zero of g / g' on the FP64 bracket (a, b), started from x0. Newton steps rotate
// the pair (sin x, cos x) by the step with a short Taylor series once the step is below
// 1e-3, so a converged polish costs one double-precision sincos. Returns the root and
// its sine and cosine.
template <bool kDeriv>
__device__ double polish_root(double a, double b, bool a_neg, double hx, double hy, double x0,
                              double& s_out, double& c_out) {
  double x = (x0 > a && x0 < b) ? x0 : 0.5 * (a + b);
  double s, c;
  sincos(x, &s, &c);
  for (int it = 0; it < 200; ++it) {
    double f, d;
    if (kDeriv) {
      f = (c * c - s * s) + hx * c + hy * s;
      d = -4.0 * s * c - hx * s + hy * c;
    } else {
      f = s * c + hx * s - hy * c;
      d = (c * c - s * s) + hx * c + hy * s;
    }
    if (f == 0.0) break;
    if ((f < 0.0) == a_neg)
      a = x;
    else
      b = x;
    const double dx = -f / d;
    if (fabs(dx) <= 2e-16 * fmax(1.0, fabs(x))) break;  // converged: x is the root
    double xn = x + dx;
    if (!(xn > a && xn < b)) {  // bisect
      xn = 0.5 * (a + b);
      if (xn == a || xn == b) break;
      x = xn;
      sincos(x, &s, &c);
      continue;
    }
    if (fabs(dx) < 1e-3) {
      const double d2 = dx * dx;
      const double cd = 1.0 - d2 * (0.5 - d2 * (1.0 / 24.0 - d2 * (1.0 / 720.0)));
      const double sd = dx * (1.0 - d2 * (1.0 / 6.0 - d2 * (1.0 / 120.0 - d2 * (1.0 / 5040.0))));
      const double cn = c * cd - s * sd;
      s = s * cd + c * sd;
      c = cn;
    } else {
      sincos(xn, &s, &c);
    }
    x = xn;
    if (fabs(dx) <= 2e-16 * fmax(1.0, fabs(x)) || (b - a) <= 4e-16 * fmax(1.0, fabs(x))) break;
  }
  s_out = s;
  c_out = c;
  return x;
}

template <bool kDeriv>
__device__ __forceinline__ double find_root(double a, double b, bool a_neg, double hx, double hy,
                                            double& s, double& c) {
  const float x0 = seed_root<kDeriv>((float)a, (float)b, a_neg, (float)hx, (float)hy);
  return polish_root<kDeriv>(a, b, a_neg, hx, hy, (double)x0, s, c);
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
  double s_c, c_c, s_o, c_o;        // sine and cosine of th_c and th_o
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
    r.s_c = r.s_o = 0.0;
    r.c_c = r.th_c == 0.0 ? 1.0 : -1.0;
    r.c_o = r.th_o == 0.0 ? 1.0 : -1.0;
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
      const double ca = sqrt((1.0 - hy) * (1.0 + hy));
      r.s_c = r.s_o = hy;
      r.c_c = toa ? ca : -ca;
      r.c_o = toa ? -ca : ca;
    } else {
      r.two = false;
      r.th_c = r.th_o = kHalfPi;
      r.e_c = r.e_o = 1.0 - 2.0 * hy;
      r.e3 = 0.0;
      r.s_c = r.s_o = 1.0;
      r.c_c = r.c_o = 0.0;
    }
    return r;
  }
  // ---- general case: reflect into hx > 0 ----
  const bool refl = hx < 0.0;
  const double ax = fabs(hx);
  double s1, c1;
  const double r1 = find_root<false>(0.0, kHalfPi, true, ax, hy, s1, c1);  // global minimum
  const double e1 = sw_energy(s1, c1, ax, hy);
  bool two = false;
  double r2a = 0.0, r2b = 0.0, e2a = 0.0, e2b = 0.0, s2 = 0.0, c2 = 0.0;
  if (astroid_bistable(ax, hy)) {
    // the zero t* of g' in (pi/2, pi) separates the saddle maximum and the metastable
    // minimum; the single-precision t* is used when g < 0 there in double precision
    double ts = (double)seed_root<true>((float)kHalfPi, (float)kPi, true, (float)ax, (float)hy);
    if (!(ts > kHalfPi && ts < kPi)) ts = 0.5 * (kHalfPi + kPi);
    double st, ct;
    sincos(ts, &st, &ct);
    if (!(st * ct + ax * st - hy * ct < 0.0)) ts = polish_root<true>(kHalfPi, kPi, true, ax, hy, ts, st, ct);
    if (st * ct + ax * st - hy * ct < 0.0) {
      two = true;
      double sa, ca;
      r2a = find_root<false>(kHalfPi, ts, false, ax, hy, sa, ca);  // saddle maximum
      r2b = find_root<false>(ts, kPi, true, ax, hy, s2, c2);       // metastable minimum
      e2a = sw_energy(sa, ca, ax, hy);
      e2b = sw_energy(s2, c2, ax, hy);
    }
  }
  // back to the unreflected frame: theta = pi - theta_r flips the cosine
  const double back1 = refl ? wrap_pi(kPi - r1) : r1;
  r.s_c = s1;
  r.c_c = refl ? -c1 : c1;
  if (!two) {
    r.two = false;
    r.th_c = r.th_o = back1;
    r.e_c = r.e_o = e1;
    r.e3 = 0.0;
    r.s_o = r.s_c;
    r.c_o = r.c_c;
    return r;
  }
  // basin of theta0. In the reflected frame the circle reads r1 (min) < r2a (max) <
  // r2b (min) < r3 (max) < r1 + 2 pi, with r3 the global maximum in (pi, 3 pi / 2);
  // r3 is only needed when the moment lies in that quadrant.
  double y = refl ? (kPi - theta0) : theta0;
  if (y >= 1.5 * kPi) y -= 2.0 * kPi;
  if (y < -kHalfPi) y += 2.0 * kPi;
  int basin;  // 1: r1, 2: r2b, 0: on a maximum
  if (y < r2a)
    basin = 1;
  else if (y == r2a)
    basin = 0;
  else if (y <= kPi)
    basin = 2;
  else {
    double s3, c3;
    const double r3 = find_root<false>(kPi, 1.5 * kPi, false, ax, hy, s3, c3);
    basin = y < r3 ? 2 : (y > r3 ? 1 : 0);
  }
  const double b2 = refl ? wrap_pi(kPi - r2b) : wrap_pi(r2b);
  if (basin == 0) {
    if (e1 != e2b) {
      basin = e1 < e2b ? 1 : 2;
    } else {
      const double d1 = fabs(wrap_pi(theta0 - back1)), d2 = fabs(wrap_pi(theta0 - b2));
      basin = ((d1 < d2) || (d1 == d2 && back1 <= b2)) ? 1 : 2;
    }
  }
  const bool to1 = basin == 1;
  const double s2u = s2, c2u = refl ? -c2 : c2;
  r.two = true;
  r.th_c = to1 ? back1 : b2;
  r.e_c = to1 ? e1 : e2b;
  r.th_o = to1 ? b2 : back1;
  r.e_o = to1 ? e2b : e1;
  r.e3 = e2a;
  r.s_c = to1 ? s1 : s2u;
  r.c_c = to1 ? (refl ? -c1 : c1) : c2u;
  r.s_o = to1 ? s2u : s1;
  r.c_o = to1 ? c2u : (refl ? -c1 : c1);
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
  double s = sw.s_c, c = sw.c_c;
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
      s = sw.s_o;
      c = sw.c_o;
      out.jump = 1;
    }
  }
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
