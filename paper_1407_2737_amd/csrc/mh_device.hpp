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

// Full 128-bit product of a 64-bit constant and x from four 32 x 32 -> 64 products,
// each with its carry-in folded into one multiply-add (none can overflow 64 bits):
// a x = ah xh 2^64 + (ah xl + al xh) 2^32 + al xl.
template <uint64_t A>
__device__ __forceinline__ void mul128(uint64_t x, uint64_t& lo, uint64_t& hi) {
  constexpr uint32_t al = (uint32_t)A, ah = (uint32_t)(A >> 32);
  const uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32);
  const uint64_t p0 = (uint64_t)al * xl;
  const uint64_t p1 = (uint64_t)al * xh + (p0 >> 32);
  const uint64_t p2 = (uint64_t)ah * xl + (uint32_t)p1;
  hi = (uint64_t)ah * xh + (p1 >> 32) + (p2 >> 32);
  lo = (p2 << 32) | (uint32_t)p0;
}

__device__ __forceinline__ void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2,
                                              uint64_t& c3, uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += kPhW0;
      k1 += kPhW1;
    }
    uint64_t lo0, hi0, lo1, hi1;
    mul128<kPhM0>(c0, lo0, hi0);
    mul128<kPhM1>(c2, lo1, hi1);
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
// Angles are carried as unit directions (sine, cosine). Brackets, Newton steps,
// bisection and the basin test then need only products and signs: the sine of the
// angle from p to q is cross(p, q), a step by dx rotates the pair, and the middle of
// an arc narrower than pi is the normalised sum of its ends. No double-precision
// sine, cosine or arctangent is evaluated on the update path.
struct Dir {
  double s, c;
};

__device__ __forceinline__ double cross(Dir p, Dir q) { return p.c * q.s - p.s * q.c; }

// 1/sqrt(x) for x > 0: hardware estimate and two Newton refinements.
__device__ __forceinline__ double rsqrt64(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  r = r * fma(-hx * r, r, 1.5);
  return r * fma(-hx * r, r, 1.5);
}

__device__ __forceinline__ Dir unit(double s, double c) {
  const double inv = rsqrt64(s * s + c * c);
  return Dir{s * inv, c * inv};
}

// Direction of the in-plane projection (p, q) = (m.u, m.n) of a moment. A zero
// projection takes the direction that atan2 gives signed zeros: angle 0 for q = +0,
// pi for q = -0.
__device__ __forceinline__ Dir dir_of(double p, double q) {
  const double rho2 = p * p + q * q;
  if (rho2 > 0.0) return unit(p, q);
  return Dir{0.0, copysign(1.0, q)};
}

__device__ __forceinline__ double sw_energy(double s, double c, double hx, double hy) {
  return s * s - 2.0 * (hx * c + hy * s);
}

// g = e'/2 (kDeriv = false) or g' = e''/2 (kDeriv = true) at direction (s, c), and its
// derivative along the angle.
template <bool kDeriv, typename T>
__device__ __forceinline__ T sw_fn(T s, T c, T hx, T hy, T& d) {
  if (kDeriv) {
    d = T(-4) * s * c - hx * s + hy * c;
    return (c * c - s * s) + hx * c + hy * s;
  }
  d = (c * c - s * s) + hx * c + hy * s;
  return s * c + hx * s - hy * c;
}

// Double-precision reciprocal for Newton steps: hardware estimate and two Newton
// refinements (the step only has to be accurate to a few ulp).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}

// FP32 seed of a zero of g / g' on the angle bracket (a, b), where the function is
// negative at a iff a_neg: Newton from x0 (the middle of the bracket when x0 is not
// inside it) kept inside the bracket, bisection when a step leaves it, stopped once a
// step is below 1e-4 rad. Returns the angle and, in (so, co), its sine and cosine with
// the last step applied to first order (about 1e-7 from the root), which is where the
// double-precision polish starts.
template <bool kDeriv>
__device__ float seed_root(float a, float b, bool a_neg, float hx, float hy, float x0,
                           float& so, float& co) {
  float x = (x0 > a && x0 < b) ? x0 : 0.5f * (a + b);
  for (int it = 0;; ++it) {
    float s, c, d;
    __sincosf(x, &s, &c);
    const float f = sw_fn<kDeriv>(s, c, hx, hy, d);
    if ((f < 0.f) == a_neg)
      a = x;
    else
      b = x;
    const float dx = -f * __builtin_amdgcn_rcpf(d);
    if (fabsf(dx) < 1e-4f) {
      so = s + c * dx;
      co = c - s * dx;
      return x + dx;
    }
    if (it == 29) {
      so = s;
      co = c;
      return x;
    }
    float xn = x + dx;
    if (!(xn > a && xn < b)) xn = 0.5f * (a + b);
    x = xn;
  }
}

// FP64 zero of g / g' on the arc (a, b) (counter-clockwise, narrower than pi), where the
// function is negative at a iff a_neg, started from direction x. Newton steps below
// 1e-3 rad rotate the direction by a short Taylor series of the step's sine and cosine;
// a step that is larger or leaves the arc is replaced by bisection. A step below 1e-12
// rad is taken and ends the polish: Newton's quadratic convergence leaves the result
// within (f''/2f') dx^2 of the root, far below the rounding of its sine and cosine
// except right at a fold. It also stops when a step below 1e-12 no longer halves
// the previous one (the iterate is inside the rounding band of the root, wide where f'
// is small) or when the arc is below 4e-16.
template <bool kDeriv>
__device__ Dir polish_root(Dir a, Dir b, bool a_neg, double hx, double hy, Dir x) {
  if (!(cross(a, x) > 0.0 && cross(x, b) > 0.0)) x = unit(a.s + b.s, a.c + b.c);
  double prev = 1.0;
  for (int it = 0; it < 200; ++it) {
    double d;
    const double f = sw_fn<kDeriv>(x.s, x.c, hx, hy, d);
    if (f == 0.0) break;
    if ((f < 0.0) == a_neg)
      a = x;
    else
      b = x;
    const double dx = -f * rcp64(d);
    const double adx = fabs(dx);
    if (adx <= 2e-16 || (adx < 1e-12 && adx > 0.5 * prev)) break;  // x is the root
    prev = adx;
    if (adx < 1e-3) {
      const double d2 = dx * dx;
      const double cd = 1.0 - d2 * (0.5 - d2 * (1.0 / 24.0 - d2 * (1.0 / 720.0)));
      const double sd = dx * (1.0 - d2 * (1.0 / 6.0 - d2 * (1.0 / 120.0 - d2 * (1.0 / 5040.0))));
      const Dir xn{x.s * cd + x.c * sd, x.c * cd - x.s * sd};
      if (cross(a, xn) > 0.0 && cross(xn, b) > 0.0) {
        x = xn;
        if (adx < 1e-12) break;
        continue;
      }
    }
    if (cross(a, b) <= 4e-16) break;
    x = unit(a.s + b.s, a.c + b.c);
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
  double e_c, e_o, e3;  // current/other minimum, lower maximum (units K V)
  double s_c, c_c, s_o, c_o;  // directions of the current and the other minimum
  bool two;
};

// Step iv-v: stationary points for (hx, hy) with hy >= 0, and the basin of the moment at
// angle theta0, given as its direction d0 = (sin theta0, cos theta0).
// ---- general case of steps iv-v, in pieces ----
// With the field reflected into hx > 0 (theta -> pi - theta flips the cosine): the
// global minimum r1; t* (the zero of g' between the saddle and the metastable minimum)
// with the two starts around it; the saddle r2a and the metastable minimum r2b; and the
// energies and basin of step v. sw_fall runs them in order; the update kernel can run
// the roots on separate waves, with the same arithmetic.
struct SWArgs {
  bool refl;       // hx < 0: reflected
  double ax, hy;   // |hx|, hy
  float axf, hyf;
};

__device__ __forceinline__ SWArgs sw_args(double hx, double hy) {
  SWArgs a;
  a.refl = hx < 0.0;
  a.ax = fabs(hx);
  a.hy = hy;
  a.axf = (float)a.ax;
  a.hyf = (float)hy;
  return a;
}

// global minimum r1 in (0, pi/2), from the FP32 start r1 = hy / (1 + hx)
__device__ __forceinline__ Dir sw_min1(const SWArgs& a) {
  const float kHalfPiF = (float)kHalfPi;
  const Dir east{0.0, 1.0}, north{1.0, 0.0};
  float fs, fc;
  seed_root<false>(0.f, kHalfPiF, true, a.axf, a.hyf, a.hyf * __builtin_amdgcn_rcpf(1.f + a.axf),
                   fs, fc);
  return polish_root<false>(east, north, true, a.ax, a.hy, unit(fs, fc));
}

struct SWT {
  bool two;   // two minima
  Dir dt;     // direction of t*
  float ts;   // t*
  float q;    // half-distance of the two starts from t*
};

// Inside the astroid: a direction between the saddle maximum and the metastable minimum
// in (pi/2, pi) (the FP32 zero t* of g' from the start 3 pi / 4 + (hx - hy) / (2 sqrt 2),
// kept when g < 0 there in double precision, else polished), and the starts
// t* -+ sqrt(-2 g / g''), the zeros of g's quadratic expansion about its minimum t*
// (exact as the pair merges at the astroid).
__device__ __forceinline__ SWT sw_tstar(const SWArgs& a) {
  const float kPiF = (float)kPi, kHalfPiF = (float)kHalfPi;
  const Dir north{1.0, 0.0}, west{0.0, -1.0};
  SWT t;
  t.two = false;
  t.dt = Dir{0.0, 0.0};
  t.ts = 0.f;
  t.q = 0.f;
  if (!astroid_bistable(a.ax, a.hy)) return t;
  const double ax = a.ax, hy = a.hy;
  const float axf = a.axf, hyf = a.hyf;
  float fs, fc;
  float ts = seed_root<true>(kHalfPiF, kPiF, true, axf, hyf,
                             0.75f * kPiF + 0.35355339f * (axf - hyf), fs, fc);
  Dir dt = unit(fs, fc);
  if (!(dt.s > 0.0 && dt.c < 0.0 && ts > kHalfPiF && ts < kPiF)) {
    ts = 0.75f * kPiF;
    dt = unit(1.0, -1.0);
  }
  double gt = dt.s * dt.c + ax * dt.s - hy * dt.c;
  if (!(gt < 0.0)) {
    dt = polish_root<true>(north, west, true, ax, hy, dt);
    gt = dt.s * dt.c + ax * dt.s - hy * dt.c;
    ts = atan2f((float)dt.s, (float)dt.c);
  }
  t.dt = dt;
  t.ts = ts;
  if (gt < 0.0) {
    t.two = true;
    float g2;
    const float st = (float)dt.s, ct = (float)dt.c;
    const float g0 = sw_fn<false>(st, ct, axf, hyf, g2);
    sw_fn<true>(st, ct, axf, hyf, g2);
    t.q = sqrtf(-2.f * g0 * __builtin_amdgcn_rcpf(g2));
  }
  return t;
}

// saddle maximum r2a in (pi/2, t*)
__device__ __forceinline__ Dir sw_saddle(const SWArgs& a, const SWT& t) {
  const float kHalfPiF = (float)kHalfPi;
  const Dir north{1.0, 0.0};
  float fs, fc;
  seed_root<false>(kHalfPiF, t.ts, false, a.axf, a.hyf, t.ts - t.q, fs, fc);
  return polish_root<false>(north, t.dt, false, a.ax, a.hy, unit(fs, fc));
}

// metastable minimum r2b in (t*, pi)
__device__ __forceinline__ Dir sw_meta(const SWArgs& a, const SWT& t) {
  const float kPiF = (float)kPi;
  const Dir west{0.0, -1.0};
  float fs, fc;
  seed_root<false>(t.ts, kPiF, true, a.axf, a.hyf, t.ts + t.q, fs, fc);
  return polish_root<false>(t.dt, west, true, a.ax, a.hy, unit(fs, fc));
}

// Step v from the roots (reflected frame): energies, the basin of theta0 (direction d0),
// and the state in the unreflected frame.
__device__ __forceinline__ SWState sw_finish(const SWArgs& a, Dir d0, Dir d1, bool two, Dir d2a,
                                             Dir d2b) {
  SWState r;
  const bool refl = a.refl;
  const double ax = a.ax, hy = a.hy;
  const double e1 = sw_energy(d1.s, d1.c, ax, hy);
  const Dir u1{d1.s, refl ? -d1.c : d1.c};  // unreflected directions
  if (!two) {
    r.two = false;
    r.e_c = r.e_o = e1;
    r.e3 = 0.0;
    r.s_c = r.s_o = u1.s;
    r.c_c = r.c_o = u1.c;
    return r;
  }
  const double e2a = sw_energy(d2a.s, d2a.c, ax, hy);
  const double e2b = sw_energy(d2b.s, d2b.c, ax, hy);
  const Dir u2{d2b.s, refl ? -d2b.c : d2b.c};
  // Basin of theta0. In the reflected frame (angle y, sine sr, cosine cr) the circle
  // reads r1 (min) < r2a (max) < r2b (min) < r3 (max) < r1 + 2 pi with r1 in (0, pi/2),
  // r2a and r2b in (pi/2, pi) and r3 in (pi, 3 pi/2):
  //   cr >= 0           y in [-pi/2, pi/2], before r2a: minimum r1;
  //   cr < 0, sr >= 0   y in (pi/2, pi]: before r2a iff sin(r2a - y) > 0;
  //   cr < 0, sr < 0    y in (pi, 3 pi/2): before r3 iff g(y) > 0, as r3 is the only
  //                     zero of g there and g(pi) = hy > 0 > -ax = g(3 pi/2).
  // A zero sine or g puts the moment on a maximum (basin 0).
  const Dir y{d0.s, refl ? -d0.c : d0.c};
  int basin;  // 1: r1, 2: r2b, 0: on a maximum
  if (y.c >= 0.0) {
    basin = 1;
  } else if (y.s >= 0.0) {
    const double x = cross(y, d2a);
    basin = x > 0.0 ? 1 : (x < 0.0 ? 2 : 0);
  } else {
    const double gy = y.s * y.c + ax * y.s - hy * y.c;
    basin = gy > 0.0 ? 2 : (gy < 0.0 ? 1 : 0);
  }
  if (basin == 0) {  // on a maximum: the lower minimum, then the nearer, then the smaller angle
    if (e1 != e2b) {
      basin = e1 < e2b ? 1 : 2;
    } else {
      const double t0 = atan2(d0.s, d0.c);
      const double t1 = atan2(u1.s, u1.c), t2 = atan2(u2.s, u2.c);
      const double dd1 = fabs(wrap_pi(t0 - t1)), dd2 = fabs(wrap_pi(t0 - t2));
      basin = ((dd1 < dd2) || (dd1 == dd2 && t1 <= t2)) ? 1 : 2;
    }
  }
  const bool to1 = basin == 1;
  r.two = true;
  r.e_c = to1 ? e1 : e2b;
  r.e_o = to1 ? e2b : e1;
  r.e3 = e2a;
  r.s_c = to1 ? u1.s : u2.s;
  r.c_c = to1 ? u1.c : u2.c;
  r.s_o = to1 ? u2.s : u1.s;
  r.c_o = to1 ? u2.c : u1.c;
  return r;
}

__device__ SWState sw_fall(double hx, double hy, Dir d0) {
  SWState r;
  // ---- exact special cases (field along or across the axis) ----
  if (hy == 0.0) {
    const double e0 = -2.0 * hx, epi = 2.0 * hx;
    bool to0;  // current minimum at theta = 0 (else pi)
    if (fabs(hx) < 1.0) {
      // maxima at +-tm with cos tm = -hx, both at energy 1 + hx^2; |theta0| < tm is
      // cos theta0 > -hx since the cosine falls on [0, pi]. On a maximum: the lower
      // minimum, then the nearer (equal here), then the smaller angle (0).
      if (d0.c > -hx)
        to0 = true;
      else if (d0.c < -hx)
        to0 = false;
      else
        to0 = e0 <= epi;
      r.two = true;
      r.e3 = 1.0 + hx * hx;
      r.e_o = to0 ? epi : e0;
    } else {
      to0 = hx > 0.0;
      r.two = false;
      r.e3 = 0.0;
      r.e_o = to0 ? e0 : epi;
    }
    r.e_c = to0 ? e0 : epi;
    r.s_c = r.s_o = 0.0;
    r.c_c = to0 ? 1.0 : -1.0;
    r.c_o = r.two ? -r.c_c : r.c_c;
    return r;
  }
  if (hx == 0.0) {
    if (hy < 1.0) {
      // minima at asin(hy) and pi - asin(hy), both at -hy^2; basins (-pi/2, pi/2) and
      // (pi/2, 3pi/2), ties (cos theta0 = 0) to the first
      const bool toa = d0.c >= 0.0;
      const double ca = sqrt((1.0 - hy) * (1.0 + hy));
      r.two = true;
      r.e_c = r.e_o = -hy * hy;
      r.e3 = 1.0 - 2.0 * hy;
      r.s_c = r.s_o = hy;
      r.c_c = toa ? ca : -ca;
      r.c_o = -r.c_c;
    } else {
      r.two = false;
      r.e_c = r.e_o = 1.0 - 2.0 * hy;
      r.e3 = 0.0;
      r.s_c = r.s_o = 1.0;
      r.c_c = r.c_o = 0.0;
    }
    return r;
  }
  const SWArgs a = sw_args(hx, hy);
  const Dir d1 = sw_min1(a);
  const SWT t = sw_tstar(a);
  Dir d2a{0.0, 0.0}, d2b{0.0, 0.0};
  if (t.two) {
    d2a = sw_saddle(a, t);
    d2b = sw_meta(a, t);
  }
  return sw_finish(a, d0, d1, t.two, d2a, d2b);
}

// Steps iv-v with step iv as the paper states it (200-point scan, Newton refinement)
// instead of the exact search of sw_fall. g = e'/2 is sampled at the 200 angles
// 2 pi j / 200 of [0, 2 pi), the value at 2 pi being the one at 0. Each sign change
// between neighbours (cyclically, the first four in grid order) marks one extremum,
// refined by Newton's method on g from the middle of its interval: at most 50 steps,
// the first one below 1e-13 being the last, the result wrapped into (-pi, pi] by the
// IEEE remainder. Products and sums are not fused here, so that the signs of g on the
// grid, which fix the number of extrema, are rounded as in plain FP64 arithmetic. A
// point is a minimum where g turns from negative to positive. Near the switching field
// a saddle and the minimum beside it can share one grid interval and are then not
// seen: the particle keeps only its stable well.
// Step v on the sorted points (ascending angle, stable): with four points the moment
// at theta0 = atan2(d0) falls into the minimum at the end of its arc, one that sits
// exactly on a maximum into the lower minimum, then the nearer; with fewer points into
// the first minimum. Kept out of line: it is selected per system at run time and is
// far heavier than sw_fall.
namespace scan200 {

struct Pt {
  double t;   // angle, or NaN
  bool mn;    // minimum
};

__device__ __forceinline__ double key(const Pt& p) { return isnan(p.t) ? INFINITY : p.t; }

__device__ __forceinline__ void order(Pt& a, Pt& b) {
  if (key(a) > key(b)) {
    const Pt t = a;
    a = b;
    b = t;
  }
}

__device__ __forceinline__ Pt at(int k, const Pt& p0, const Pt& p1, const Pt& p2,
                                 const Pt& p3) {
  return k == 0 ? p0 : (k == 1 ? p1 : (k == 2 ? p2 : p3));
}

__device__ __forceinline__ double refine(double x, double hx, double hy) {
#pragma clang fp contract(off)
  for (int it = 0; it < 50; ++it) {
    double s, c;
    sincos(x, &s, &c);
    const double f = s * c + hx * s - hy * c;
    const double d = (c * c - s * s) + hx * c + hy * s;
    const double dx = f / d;
    x -= dx;
    if (fabs(dx) < 1e-13) break;
  }
  const double r = remainder(x, 2.0 * kPi);
  return r == -kPi ? kPi : r;
}

__device__ __forceinline__ double energy_at(double t, double hx, double hy) {
#pragma clang fp contract(off)
  double s, c;
  sincos(isnan(t) ? 0.0 : t, &s, &c);
  return s * s - 2.0 * (hx * c + hy * s);
}

}  // namespace scan200

__device__ __noinline__ SWState sw_fall_scan200(double hx, double hy, Dir d0) {
#pragma clang fp contract(off)
  using namespace scan200;
  Pt p0{NAN, false}, p1{NAN, false}, p2{NAN, false}, p3{NAN, false};
  int cnt = 0;
  double s, c;
  sincos(0.0, &s, &c);
  const bool neg0 = s * c + hx * s - hy * c < 0.0;
  bool neg_prev = neg0;
  double t_prev = 0.0;
  for (int j = 1; j <= 200; ++j) {
    const double t = 2.0 * kPi * (double)j / 200.0;
    bool neg = neg0;
    if (j < 200) {
      sincos(t, &s, &c);
      neg = s * c + hx * s - hy * c < 0.0;
    }
    if (neg != neg_prev && cnt < 4) {
      const Pt q{refine(0.5 * (t_prev + t), hx, hy), neg_prev};
      if (cnt == 0) p0 = q;
      if (cnt == 1) p1 = q;
      if (cnt == 2) p2 = q;
      if (cnt == 3) p3 = q;
      ++cnt;
    }
    neg_prev = neg;
    t_prev = t;
  }
  // stable sort by angle (adjacent exchanges on strict order), NaN last
  order(p0, p1);
  order(p1, p2);
  order(p2, p3);
  order(p0, p1);
  order(p1, p2);
  order(p0, p1);
  const double e0 = energy_at(p0.t, hx, hy), e1 = energy_at(p1.t, hx, hy);
  const double e2 = energy_at(p2.t, hx, hy), e3 = energy_at(p3.t, hx, hy);
  auto energy_of = [&](int k) { return k == 0 ? e0 : (k == 1 ? e1 : (k == 2 ? e2 : e3)); };
  const bool two = cnt == 4;
  int ic, io;
  if (!two) {
    const bool v0 = p0.mn && !isnan(p0.t), v1 = p1.mn && !isnan(p1.t);
    const bool v2 = p2.mn && !isnan(p2.t), v3 = p3.mn && !isnan(p3.t);
    ic = v0 ? 0 : (v1 ? 1 : (v2 ? 2 : (v3 ? 3 : 0)));
    io = ic;
  } else {
    const double t0 = atan2(d0.s, d0.c);
    const int j = (p0.t < t0) + (p1.t < t0) + (p2.t < t0) + (p3.t < t0);
    const int left = (j + 3) & 3, right = j & 3;
    ic = at(left, p0, p1, p2, p3).mn ? left : right;
    int hit = -1;
    if (p3.t == t0) hit = 3;
    if (p2.t == t0) hit = 2;
    if (p1.t == t0) hit = 1;
    if (p0.t == t0) hit = 0;
    // the two minima in slot order
    const int ma = p0.mn ? 0 : (p1.mn ? 1 : (p2.mn ? 2 : 3));
    const int mb = p3.mn ? 3 : (p2.mn ? 2 : (p1.mn ? 1 : 0));
    if (hit >= 0) {
      if (at(hit, p0, p1, p2, p3).mn) {
        ic = hit;
      } else if (energy_of(ma) != energy_of(mb)) {
        ic = energy_of(ma) < energy_of(mb) ? ma : mb;
      } else {
        const double da = fabs(wrap_pi(t0 - at(ma, p0, p1, p2, p3).t));
        const double db = fabs(wrap_pi(t0 - at(mb, p0, p1, p2, p3).t));
        ic = da <= db ? ma : mb;
      }
    }
    io = ic == ma ? mb : ma;
  }
  SWState r;
  r.two = two;
  const double tc = at(ic, p0, p1, p2, p3).t, to = at(io, p0, p1, p2, p3).t;
  sincos(isnan(tc) ? 0.0 : tc, &r.s_c, &r.c_c);
  sincos(isnan(to) ? 0.0 : to, &r.s_o, &r.c_o);
  r.e_c = energy_of(ic);
  r.e_o = energy_of(io);
  r.e3 = NAN;
  if (two) {
    double lo = INFINITY;
    if (!p0.mn) lo = fmin(lo, e0);
    if (!p1.mn) lo = fmin(lo, e1);
    if (!p2.mn) lo = fmin(lo, e2);
    if (!p3.mn) lo = fmin(lo, e3);
    r.e3 = lo;
  }
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
  int scan200;      // step iv as the 200-point scan (sw_fall_scan200), else the exact search
  int thermal;      // T > 0
  int aniso;        // K > 0
};

struct NPResult {
  double mx, my, mz;
  double P;
  int jump;
  int two;
};

// Step iii: the working plane (n, u) of a particle with axis n in the field B, the
// reduced in-plane field (hx, hy) and the direction of the moment m in that plane.
// When B has no component across the axis (|B_perp| <= 1e-12 max(|B|, mu0 H_K),
// compared in squares) u is the unit part of m across the axis, else n x e with e the
// coordinate axis least aligned with n (first on ties); deg marks that case.
struct Plane {
  double ux, uy, uz, hx, hy;
  Dir d0;
  bool deg;
};

__device__ __forceinline__ Plane working_plane(const NPParams& p, double Bx, double By, double Bz,
                                               double nx, double ny, double nz, double mx,
                                               double my, double mz) {
  Plane w;
  const double bpar = Bx * nx + By * ny + Bz * nz;
  double px = Bx - bpar * nx, py = By - bpar * ny, pz = Bz - bpar * nz;
  const double bp2 = px * px + py * py + pz * pz;
  const double bn2 = Bx * Bx + By * By + Bz * Bz;
  w.deg = !(bp2 > 1e-24 * fmax(bn2, p.BK * p.BK));
  if (!w.deg) {
    const double inv = rsqrt64(bp2);
    w.ux = px * inv;
    w.uy = py * inv;
    w.uz = pz * inv;
    w.hy = bp2 * inv * p.BK_inv;
  } else {
    w.hy = 0.0;
    const double mn = mx * nx + my * ny + mz * nz;
    double vx = mx - mn * nx, vy = my - mn * ny, vz = mz - mn * nz;
    const double vn = sqrt(vx * vx + vy * vy + vz * vz);
    if (vn > 1e-12) {
      w.ux = vx / vn;
      w.uy = vy / vn;
      w.uz = vz / vn;
    } else {
      const double ax = fabs(nx), ay = fabs(ny), az = fabs(nz);
      int c = 0;
      if (ay < ax) c = 1;
      if (az < (c == 0 ? ax : ay)) c = 2;
      const double ex = c == 0, ey = c == 1, ez = c == 2;
      vx = ny * ez - nz * ey;
      vy = nz * ex - nx * ez;
      vz = nx * ey - ny * ex;
      const double wn = sqrt(vx * vx + vy * vy + vz * vz);
      w.ux = vx / wn;
      w.uy = vy / wn;
      w.uz = vz / wn;
    }
  }
  w.hx = bpar * p.BK_inv;
  w.d0 = dir_of(mx * w.ux + my * w.uy + mz * w.uz, mx * nx + my * ny + mz * nz);
  return w;
}

// Eq. 5 for both directions between the wells c and o (a = barrier / k_B T): P_co
// to leave c for o and P_oc the reverse. sigma = 1 / (1 + e^(a_c - a_o)) is formed as
// e^-a_c / (e^-a_c + e^-a_o). Below kSumMin the reciprocal of that sum would overflow
// (a subnormal sum); both probabilities are then at most nu0 dt kSumMin, below any
// nonzero draw (2^-53), and are returned as 0. The single-rate form is
// -expm1(-nu0 dt e^-a).
constexpr double kSumMin = 0x1p-1000;

__device__ __forceinline__ void transition_pair(const NPParams& p, double a_c, double a_o,
                                                double& P_co, double& P_oc) {
  const double xc = exp(-a_c), xo = exp(-a_o);
  if (p.prob_form == 1) {
    P_co = -expm1(-p.nu0dt * xc);
    P_oc = -expm1(-p.nu0dt * xo);
    return;
  }
  const double sum = xc + xo;
  if (!(sum >= kSumMin)) {
    P_co = P_oc = 0.0;
    return;
  }
  const double r = rcp64(sum), q = -expm1(-p.nu0dt * sum);
  P_co = (xc * r) * q;
  P_oc = (xo * r) * q;
}

__device__ __forceinline__ NPResult np_finish(const NPParams& p, const Plane& w,
                                              const SWState& sw, double nx, double ny,
                                              double nz, uint64_t seed, uint64_t stream,
                                              int64_t i, int64_t k);

// kScan: the kernel also serves systems whose step iv is the 200-point scan (p.scan200);
// without it that search is not compiled in, so the exact path keeps its registers.
template <bool kScan = false>
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
  // step iii
  const Plane w = working_plane(p, Bx, By, Bz, nx, ny, nz, mx, my, mz);
  // steps iv-v
  const SWState sw = (kScan && p.scan200) ? sw_fall_scan200(w.hx, w.hy, w.d0)
                                          : sw_fall(w.hx, w.hy, w.d0);
  return np_finish(p, w, sw, nx, ny, nz, seed, stream, i, k);
}

// Steps vi-vii and the new moment, from the working plane and the fall (K > 0); draw()
// gives the particle's uniform number of the step, called only where two minima exist
// at T > 0.
template <typename Draw>
__device__ __forceinline__ NPResult np_finish_with(const NPParams& p, const Plane& w,
                                                   const SWState& sw, double nx, double ny,
                                                   double nz, Draw&& draw) {
  NPResult out;
  out.P = 0.0;
  out.jump = 0;
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
      // sigma = 1 / (1 + e^(a_c - a_o)) = e^-a_c / (e^-a_c + e^-a_o); below kSumMin
      // P is at most nu0 dt kSumMin and is taken as 0 (see transition_pair)
      const double xc = exp(-a_c), xo = exp(-a_o), sum = xc + xo;
      P = sum >= kSumMin ? (xc * rcp64(sum)) * (-expm1(-p.nu0dt * sum)) : 0.0;
    }
    const double u = draw();
    out.P = P;
    if (u < P) {
      s = sw.s_o;
      c = sw.c_o;
      out.jump = 1;
    }
  }
  out.mx = c * nx + s * w.ux;
  out.my = c * ny + s * w.uy;
  out.mz = c * nz + s * w.uz;
  return out;
}

__device__ __forceinline__ NPResult np_finish(const NPParams& p, const Plane& w,
                                              const SWState& sw, double nx, double ny,
                                              double nz, uint64_t seed, uint64_t stream,
                                              int64_t i, int64_t k) {
  return np_finish_with(p, w, sw, nx, ny, nz,
                        [&] { return philox_uniform(seed, stream, i, k); });
}

// Mean-magnetisation (master-equation) state of one non-interacting particle: two
// weighted moments, wells A and B (Sec. II.3, the paper's validation method).
struct MasterState {
  double ax, ay, az, bx, by, bz, wa, wb;
};

__device__ __forceinline__ void master_init(MasterState& q, double nx, double ny, double nz,
                                            double ex, double ey, double ez) {
  const double sg = nx * ex + ny * ey + nz * ez >= 0.0 ? 1.0 : -1.0;
  q.ax = q.bx = sg * nx;
  q.ay = q.by = sg * ny;
  q.az = q.bz = sg * nz;
  q.wa = 1.0;
  q.wb = 0.0;
}

// One step in the applied field Bext e_H: both weighted moments fall (steps iii-v; B
// uses A's plane unless the field lies along the axis, where the plane follows each
// moment and the minima are +-n), weights reaching the same minimum are pooled, Eq. 5
// moves w_c P(c->o) from each well to the other (steps vi-vii), and with one minimum
// all weight goes to it. Requires K > 0. Returns the expected moment along e_H.
__device__ __forceinline__ double master_step(const NPParams& p, double Bext, double ex,
                                              double ey, double ez, double nx, double ny,
                                              double nz, MasterState& q) {
  const double Bx = Bext * ex, By = Bext * ey, Bz = Bext * ez;
  const Plane pa = working_plane(p, Bx, By, Bz, nx, ny, nz, q.ax, q.ay, q.az);
  const SWState fa = sw_fall(pa.hx, pa.hy, pa.d0);
  Plane pb = pa;
  if (pa.deg)
    pb = working_plane(p, Bx, By, Bz, nx, ny, nz, q.bx, q.by, q.bz);
  else
    pb.d0 = dir_of(q.bx * pa.ux + q.by * pa.uy + q.bz * pa.uz, q.bx * nx + q.by * ny + q.bz * nz);
  const SWState fb = sw_fall(pb.hx, pb.hy, pb.d0);
  // the same (hx, hy) give bitwise the same minima, so the pooling test is exact
  const bool same = fb.s_c == fa.s_c && fb.c_c == fa.c_c;
  double w1 = q.wa + (same ? q.wb : 0.0), w2 = same ? 0.0 : q.wb;
  if (!fa.two) {
    w1 = 1.0;
    w2 = 0.0;
  } else if (p.thermal) {
    double P12, P21;
    transition_pair(p, p.beta * (fa.e3 - fa.e_c), p.beta * (fa.e3 - fa.e_o), P12, P21);
    const double n1 = w1 * (1.0 - P12) + w2 * P21;
    const double n2 = w2 * (1.0 - P21) + w1 * P12;
    w1 = n1;
    w2 = n2;
  }
  q.ax = fa.c_c * nx + fa.s_c * pa.ux;
  q.ay = fa.c_c * ny + fa.s_c * pa.uy;
  q.az = fa.c_c * nz + fa.s_c * pa.uz;
  q.bx = fa.c_o * nx + fa.s_o * pa.ux;
  q.by = fa.c_o * ny + fa.s_o * pa.uy;
  q.bz = fa.c_o * nz + fa.s_o * pa.uz;
  q.wa = w1;
  q.wb = w2;
  return w1 * (q.ax * ex + q.ay * ey + q.az * ez) + w2 * (q.bx * ex + q.by * ey + q.bz * ez);
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
