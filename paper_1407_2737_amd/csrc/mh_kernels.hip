// Fused kMC step kernels for gfx950 (Tan, Carrey and Respaud, arXiv:1407.2737,
// Sec. II.1 steps i-viii).
//
// Every step does, for every particle of every system (assembly x replica):
//   ii   the exact dipolar field of Eq. 1 from the start-of-step moments,
//   iii-v the working plane, Stoner-Wohlfarth extrema (Eq. 2) and the fall,
//   vi-vii the two-state switching draw (Eqs. 3-5) from a Philox stream,
// then writes the moment into the other half of a double buffer (all particles move
// synchronously from the start-of-step state, Sec. II.2) and accumulates the
// per-particle loop area and the loop record of the kept periods.
//
// Two launch forms of the same step:
//   k_resident  one workgroup owns a whole small system and runs every step in one
//               launch, positions and field-side moments resident in LDS;
//   k_field +   two launches per step: the dipolar sums over (system, i-tile) blocks
//   k_update    with sources staged through LDS, then one thread per particle for
//               the per-particle update (k_update3 for launches of few blocks: the
//               roots of the fall on three waves per particle, same results).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mh_kernels.hpp"

namespace mh {

template <typename T>
struct V4;
template <>
struct V4<double> {
  using type = D4;
};
template <>
struct V4<float> {
  using type = F4;
};

template <typename T>
__device__ __forceinline__ const typename V4<T>::type* pos_of(const SysDesc& s);
template <>
__device__ __forceinline__ const D4* pos_of<double>(const SysDesc& s) {
  return s.pos64;
}
template <>
__device__ __forceinline__ const F4* pos_of<float>(const SysDesc& s) {
  return s.pos32;
}
template <typename T>
__device__ __forceinline__ typename V4<T>::type* mom_of(const SysDesc& s);
template <>
__device__ __forceinline__ D4* mom_of<double>(const SysDesc& s) {
  return s.m64;
}
template <>
__device__ __forceinline__ F4* mom_of<float>(const SysDesc& s) {
  return s.m32;
}

// 1/r for a squared distance in units of d. Distinct particles are at least one
// diameter apart and padding sits at 1e15, so r2 is 0 (the pair j == i, masked by the
// caller) or a normal number: the hardware reciprocal square root needs none of the
// subnormal scaling that rsqrtf wraps around it. In FP64 its estimate is refined by two
// Newton steps (rsqrt64), in place of a square root and a division.
__device__ __forceinline__ float rsqrt_dist(float r2) { return __builtin_amdgcn_rsqf(r2); }
__device__ __forceinline__ double rsqrt_dist(double r2) { return rsqrt64(r2); }

// Eq. 1 term of source j on target i in reduced units (positions / d): accumulates
// (3 (m.r) r / r^2 - m) / r^3 with r = p_j - p_i; a coincident pair (j == i)
// contributes nothing.
template <typename T, bool kGuard = true, typename P4, typename M4>
__device__ __forceinline__ void dip_pair(T xi, T yi, T zi, const P4& pj, const M4& mj, T& bx,
                                         T& by, T& bz) {
  const T dx = (T)pj.x - xi, dy = (T)pj.y - yi, dz = (T)pj.z - zi;
  const T r2 = dx * dx + dy * dy + dz * dz;
  T inv = rsqrt_dist(r2);
  if constexpr (kGuard) inv = r2 > (T)0 ? inv : (T)0;
  const T inv2 = inv * inv;
  const T inv3 = inv2 * inv;
  const T md = (T)mj.x * dx + (T)mj.y * dy + (T)mj.z * dz;
  const T s = (T)3 * md * inv2;
  bx += inv3 * (s * dx - (T)mj.x);
  by += inv3 * (s * dy - (T)mj.y);
  bz += inv3 * (s * dz - (T)mj.z);
}

// Fixed-order block sum of one double per thread (blockDim.x == 256).
__device__ __forceinline__ double block_sum_256(double v, double* red) {
  const int tid = threadIdx.x;
  v = wave_sum(v);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  const double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------------------
// Resident form: one workgroup of kResThreads threads per system, steps [k0, k1).
// Dynamic LDS: pos[nmax] then mom[2][nmax] (field precision T).
// ---------------------------------------------------------------------------
// Threads of a resident workgroup. Fixed, so that a system's results do not depend on
// the launch it is part of: 512 threads halved the latency of the pair sums of small
// systems (N = 100: 16.0 -> 14.2 us per step) but, with the update on one thread per
// particle, cost 23 % of the throughput of many systems at once.
constexpr int kResThreads = 256;
static_assert(kResThreads / 64 == kRecSlots, "one loop-record slot per resident wave");

// Fixed-order sum of one double per thread over a kResThreads block: wave sums, then a
// pairwise tree over the waves.
__device__ __forceinline__ double block_sum_res(double v, double* red) {
  const int tid = threadIdx.x;
  v = wave_sum(v);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double w[kResThreads / 64];
#pragma unroll
  for (int q = 0; q < kResThreads / 64; ++q) w[q] = red[q];
#pragma unroll
  for (int h = kResThreads / 128; h > 0; h >>= 1)
#pragma unroll
    for (int q = 0; q < h; ++q) w[q] = w[2 * q] + w[2 * q + 1];
  __syncthreads();
  return w[0];
}

template <typename T, bool kScan>
__global__ __launch_bounds__(kResThreads) void k_resident(const SysDesc* __restrict__ systems,
                                                          int64_t k0, int64_t k1, int nmax) {
  using P4 = typename V4<T>::type;
  extern __shared__ __align__(32) unsigned char smem[];
  P4* pos = reinterpret_cast<P4*>(smem);
  P4* mom = pos + nmax;
  __shared__ double red[kResThreads / 64];
  const SysDesc s = systems[blockIdx.x];
  const int n = s.n;
  const int tid = threadIdx.x;
  const P4* gpos = pos_of<T>(s);
  const P4* gmom = mom_of<T>(s);
  // local step range of this system within the launch's global range
  const int64_t kl0 = k0 - s.k_origin > 0 ? k0 - s.k_origin : 0;
  const int64_t kl1 = k1 - s.k_origin < (int64_t)s.total_steps ? k1 - s.k_origin : s.total_steps;
  if (kl0 >= kl1) return;
  const int cur0 = (int)(kl0 & 1);
  for (int j = tid; j < n; j += kResThreads) {
    pos[j] = gpos[j];
    mom[(int64_t)cur0 * nmax + j] = gmom[(int64_t)cur0 * s.stride + j];
  }
  // threads per particle: largest power of two with P * n <= kResThreads, at most 64
  int P = 1;
  while (P < 64 && 2 * P * n <= kResThreads) P *= 2;
  const int per_pass = kResThreads / P;
  const int sub = tid % P;
  // A system that takes one pass per step gives each updating thread the same particle
  // in every step: its axis and area accumulator are held in registers for the whole
  // launch, its FP64 moment is read from the LDS copy (FP64 systems) and the new one is
  // written there from registers, so the step's chain makes no global memory round trip
  // (the state in memory is written as before; field-only evaluations, whose
  // descriptors may carry no area buffer, keep the general path).
  const int i_own = tid / P;
  const bool own = n <= per_pass && sub == 0 && i_own < n && !s.field_only;
  D4 nn_own = {0.0, 0.0, 0.0, 0.0};
  double acc[2] = {0.0, 0.0};
  if (own) {
    nn_own = s.axes[i_own];
    acc[0] = s.area[i_own];
    acc[1] = s.area[n + i_own];
  }
  __syncthreads();
  for (int64_t k = kl0; k < kl1; ++k) {
    const int cur = (int)(k & 1);
    const P4* mc = mom + (int64_t)cur * nmax;
    double mxsum = 0.0;
    for (int base = 0; base < n; base += per_pass) {
      const int i = base + tid / P;
      T bx = 0, by = 0, bz = 0;
      if (i < n) {
        const P4 pi = pos[i];
        if (s.Bscale != 0.0) {  // interactions on (uniform over the block)
          // two pairs per trip into separate sums, so that their LDS reads and FP64
          // chains overlap (one workgroup per system: the step is latency-bound)
          T cx = 0, cy = 0, cz = 0;
          int j = sub;
          for (; j + P < n; j += 2 * P) {
            dip_pair<T>((T)pi.x, (T)pi.y, (T)pi.z, pos[j], mc[j], bx, by, bz);
            dip_pair<T>((T)pi.x, (T)pi.y, (T)pi.z, pos[j + P], mc[j + P], cx, cy, cz);
          }
          if (j < n) dip_pair<T>((T)pi.x, (T)pi.y, (T)pi.z, pos[j], mc[j], bx, by, bz);
          bx += cx;
          by += cy;
          bz += cz;
        }
      }
      for (int off = P >> 1; off > 0; off >>= 1) {
        bx += __shfl_xor(bx, off, 64);
        by += __shfl_xor(by, off, 64);
        bz += __shfl_xor(bz, off, 64);
      }
      if (own) {  // (one pass: i == i_own)
        D4 mo;
        if constexpr (sizeof(T) == 8) {
          const P4 ml = mc[i];
          mo = D4{ml.x, ml.y, ml.z, 0.0};
        } else {
          mo = ldg(s.m64 + (int64_t)cur * s.stride + i);
        }
        D4 mn;
        mxsum += np_epilogue<kScan>(s, i, k, cur, (double)bx, (double)by, (double)bz,
                                    NPState{mo, nn_own}, acc, &mn);
        P4 v;
        v.x = mn.x;
        v.y = mn.y;
        v.z = mn.z;
        v.w = 0;
        mom[(int64_t)(cur ^ 1) * nmax + i] = v;
      } else if (i < n && sub == 0) {
        const double mx = np_epilogue<kScan>(s, i, k, cur, (double)bx, (double)by, (double)bz);
        mxsum += mx;
        if (s.field_only) continue;
        const D4 m = s.m64[(int64_t)(cur ^ 1) * s.stride + i];
        P4 v;
        v.x = m.x;
        v.y = m.y;
        v.z = m.z;
        v.w = 0;
        mom[(int64_t)(cur ^ 1) * nmax + i] = v;
      }
    }
    __syncthreads();
    if (k >= s.kept0 && !s.field_only) {
      if (s.rec_slots == kRecSlots) {  // one slot per wave: no block reduction, no barrier
        double v = mxsum;
        v = wave_sum(v);
        if ((tid & 63) == 0) s.recpart[(k - s.kept0) * kRecSlots + (tid >> 6)] = v;
      } else {
        const double tot = block_sum_res(mxsum, red);
        if (tid == 0) s.recpart[k - s.kept0] = tot;
      }
    }
  }
}

// Latency floor of a resident step: kResThreads threads pass one value each through a
// double-buffered LDS array across one barrier per step, as a resident step passes the
// moments to the next step's sums; the last value goes to sink so that nothing is
// optimised away.
__global__ __launch_bounds__(kResThreads) void k_empty_steps(int64_t steps, double* sink) {
  __shared__ double v[2][kResThreads];
  const int t = threadIdx.x;
  double a = (double)t;
  v[0][t] = a;
  __syncthreads();
  for (int64_t k = 0; k < steps; ++k) {
    const int cur = (int)(k & 1);
    a += v[cur][(t + 1) % kResThreads];
    v[cur ^ 1][t] = a;
    __syncthreads();
  }
  if (t == 0) sink[0] = a;
}

// ---------------------------------------------------------------------------
// Tiled form: two launches per step k.
//
// Pairs (target, q + it Q), it < ce / Q, of one staged chunk; with G > 1 the pair
// geometry is shared by the G replicas' moments; kGuard masks the pair j == i. The trip
// count is the same for every lane (ce is a multiple of Q and q < Q), so the loop runs
// on a scalar counter, and a full chunk of at most 16 trips is unrolled whole, which
// makes every LDS offset an immediate: no per-pair VALU work but the pair terms.
template <typename T, int G, bool kGuard, int Q, int CH, typename P4>
__device__ __forceinline__ void chunk_pairs(int q, int ce, T xi, T yi, T zi, const P4* spos,
                                            const P4 (*smom)[CH], T* bx, T* by, T* bz) {
  auto pair = [&](int e) {
    if constexpr (G == 1) {
      dip_pair<T, kGuard>(xi, yi, zi, spos[e], smom[0][e], bx[0], by[0], bz[0]);
    } else {
      const P4 pj = spos[e];
      const T dx = (T)pj.x - xi, dy = (T)pj.y - yi, dz = (T)pj.z - zi;
      const T r2 = dx * dx + dy * dy + dz * dz;
      T inv = rsqrt_dist(r2);
      if constexpr (kGuard) inv = r2 > (T)0 ? inv : (T)0;
      const T inv2 = inv * inv;
      const T inv3 = inv2 * inv;
      const T s3 = (T)3 * inv2;
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const P4 mj = smom[r][e];
        const T md = ((T)mj.x * dx + (T)mj.y * dy + (T)mj.z * dz) * s3;
        bx[r] += inv3 * (md * dx - (T)mj.x);
        by[r] += inv3 * (md * dy - (T)mj.y);
        bz[r] += inv3 * (md * dz - (T)mj.z);
      }
    }
  };
  if (CH / Q <= 16 && ce == CH) {
#pragma unroll
    for (int it = 0; it < CH / Q; ++it) pair(q + it * Q);
  } else {
    const int nit = ce / Q;
#pragma unroll 2
    for (int it = 0; it < nit; ++it) pair(q + it * Q);
  }
}

// k_field over (system, i-tile) blocks of 1024 threads. A block owns TI targets; its
// 16 waves split the sources into Q = 16 * 64 / TI interleaved streams (lane l of wave
// w: target l % TI, stream w * (64/TI) + l / TI). Sources are staged through LDS in
// chunks of CH; partial fields are then reduced across streams in LDS, which reuses the
// staging space, in a fixed two-level order in FP64 (sums of 16 streams, then of those
// sums) and written per particle. No block depends on another.
//
// k_update, one thread per particle: steps iii-vii and the accumulations.
// ---------------------------------------------------------------------------
template <typename T, int TI, int G>
// At most 64 VGPRs where the unrolled loop allows it, so that two blocks share a CU.
__global__ __launch_bounds__(1024, 8) void k_field(const SysDesc* __restrict__ systems,
                                                const int4* __restrict__ tiles,
                                                const int64_t* __restrict__ kbase, int64_t koff) {
  using P4 = typename V4<T>::type;
  constexpr int L = 64 / TI;                       // streams per wave
  constexpr int Q = 16 * L;                        // streams per block
  constexpr int CH = G <= 3 ? 1024 : 512;          // sources per staged chunk
  constexpr int NPART = Q / 16;                    // first-level sums of 16 streams
  constexpr size_t kStage = sizeof(P4) * CH * (1 + G);
  constexpr int TIP = TI + 1;  // stream rows padded: the 16-stream groups on distinct banks
  constexpr size_t kRed = sizeof(T) * 3 * G * Q * TIP;
  constexpr size_t kPart = sizeof(double) * 3 * G * NPART * TI;
  constexpr size_t kRedEnd = (kRed + 7) / 8 * 8 + kPart;
  constexpr size_t kLds = kStage > kRedEnd ? kStage : kRedEnd;
  static_assert(Q % 16 == 0, "stream layout");
  __shared__ __align__(16) unsigned char lds[kLds];
  P4* spos = reinterpret_cast<P4*>(lds);                           // staged chunk
  P4 (*smom)[CH] = reinterpret_cast<P4 (*)[CH]>(lds + sizeof(P4) * CH);
  T (*red)[G][Q][TIP] = reinterpret_cast<T (*)[G][Q][TIP]>(lds);   // after the last chunk
  double (*part)[G][NPART][TI] =
      reinterpret_cast<double (*)[G][NPART][TI]>(lds + (kRed + 7) / 8 * 8);
  const int4 tlv = tiles[blockIdx.x];  // (first system, i-tile, replicas, part), uniform
  const int4 tl = make_int4(__builtin_amdgcn_readfirstlane(tlv.x), __builtin_amdgcn_readfirstlane(tlv.y),
                            __builtin_amdgcn_readfirstlane(tlv.z), __builtin_amdgcn_readfirstlane(tlv.w));
  const int64_t kb0 = step_base(kbase, systems);
  const SysDesc& s = systems[tl.x];
  // with the prefetched fields, what the first staging loads need, in the same batch:
  // positions, field scale and the moment buffers of the block's replicas
  const P4* gpos = pos_of<T>(s);
  const double bscale = s.Bscale;
  const P4* gm0[G];
#pragma unroll
  for (int r = 0; r < G; ++r) gm0[r] = mom_of<T>(systems[tl.x + (r < tl.z ? r : 0)]);
  desc_prefetch(s, gpos, gm0[0], G > 1 ? gm0[G > 1 ? 1 : 0] : nullptr,
                G > 2 ? gm0[G > 2 ? 2 : 0] : nullptr, G > 3 ? gm0[G > 3 ? 3 : 0] : nullptr, bscale);
  const int64_t k = kb0 + koff - s.k_origin;  // local step
  if (k < 0 || k >= s.total_steps) return;
  const int n = s.n;
  const int gn = tl.z;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int il = l % TI;
  const int q = w * L + l / TI;
  const int i = tl.y * TI + il;
  const int cur = (int)(k & 1);
  const P4* gmom[G];
#pragma unroll
  for (int r = 0; r < G; ++r) gmom[r] = gm0[r] + (int64_t)cur * s.stride;
  T bx[G], by[G], bz[G];
#pragma unroll
  for (int r = 0; r < G; ++r) bx[r] = by[r] = bz[r] = (T)0;
  // sources of this block: part tl.w of nsplit equal parts (multiples of Q)
  const int per = ((n + s.nsplit - 1) / s.nsplit + Q - 1) / Q * Q;
  const int jb = tl.w * per, je = min(n, jb + per);
  if (bscale != 0.0 && n > 1) {
    const P4 pi = gpos[i < n ? i : n - 1];
    const T xi = (T)pi.x, yi = (T)pi.y, zi = (T)pi.z;
    for (int c0 = jb; c0 < je; c0 += CH) {
      const int cn = min(CH, je - c0);
      __syncthreads();
      for (int j = tid; j < CH; j += 1024) {
        // all loads first (padding entries read the chunk's last source), then the masks,
        // so that the global loads are in flight together
        const bool in = j < cn;
        const int src = c0 + (in ? j : cn - 1);
        P4 p = ldg(gpos + src);
        P4 m[G];
#pragma unroll
        for (int r = 0; r < G; ++r) m[r] = ldg(gmom[r] + src);
        // padding: far away and without moment, contributes exactly zero. The masks are
        // arithmetic (finite data times 0 or 1) so that the loads stay unconditional.
        const T keep = in ? (T)1 : (T)0, far = in ? (T)0 : (T)1e15;
        p.x = p.x * keep + far;
        p.y = p.y * keep + far;
        p.z = p.z * keep + far;
        p.w = p.w * keep;
        spos[j] = p;
#pragma unroll
        for (int r = 0; r < G; ++r) {
          const T mk = r < gn ? keep : (T)0;
          m[r].x *= mk;
          m[r].y *= mk;
          m[r].z *= mk;
          m[r].w *= mk;
          smom[r][j] = m[r];
        }
      }
      __syncthreads();
      const int ce = (cn + Q - 1) / Q * Q;  // streams stay in lockstep over padded entries
      // only the chunk holding this block's targets can contain j == i
      const bool self = (tl.y * TI < c0 + cn) && (tl.y * TI + TI > c0);
      if (self)
        chunk_pairs<T, G, true, Q, CH>(q, ce, xi, yi, zi, spos, smom, bx, by, bz);
      else
        chunk_pairs<T, G, false, Q, CH>(q, ce, xi, yi, zi, spos, smom, bx, by, bz);
    }
  }
  __syncthreads();  // every read of the staged chunk is done before red overwrites it
#pragma unroll
  for (int r = 0; r < G; ++r) {
    red[0][r][q][il] = bx[r];
    red[1][r][q][il] = by[r];
    red[2][r][q][il] = bz[r];
  }
  __syncthreads();
  // fixed-order FP64 reduction over the streams: thread (c, r, p, t) adds streams
  // 16 p .. 16 p + 15, then thread (r, t) adds the NPART sums
  if (tid < 3 * G * NPART * TI) {
    const int t = tid % TI, pp = (tid / TI) % NPART, r = (tid / (TI * NPART)) % G;
    const int c = tid / (TI * NPART * G);
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) acc += (double)red[c][r][pp * 16 + u][t];
    part[c][r][pp][t] = acc;
  }
  __syncthreads();
  if (tid < G * TI) {
    const int r = tid / TI, t = tid % TI;
    const int ii = tl.y * TI + t;
    if (r < gn && ii < n) {
      double ax = 0, ay = 0, az = 0;
#pragma unroll
      for (int pp = 0; pp < NPART; ++pp) {
        ax += part[0][r][pp][t];
        ay += part[1][r][pp][t];
        az += part[2][r][pp][t];
      }
      // the part's sum, FP32 for the FP32 field form (the update adds parts in FP64)
      P4 f;
      f.x = (T)ax;
      f.y = (T)ay;
      f.z = (T)az;
      f.w = (T)0;
      if constexpr (sizeof(T) == 4)
        systems[tl.x + r].field32[(int64_t)tl.w * n + ii] = f;
      else
        systems[tl.x + r].field[(int64_t)tl.w * n + ii] = f;
    }
  }
}

template <bool kScan>
__global__ __launch_bounds__(256) void k_update(const SysDesc* __restrict__ systems,
                                                const int2* __restrict__ blocks,
                                                const int64_t* __restrict__ kbase, int64_t koff) {
  __shared__ double red[4];
  // the block's (system, particle block) is uniform: keep it in scalar registers, so the
  // descriptor is read with scalar loads and data loads are not chained behind it
  const int2 blv = blocks[blockIdx.x];
  const int2 bl = make_int2(__builtin_amdgcn_readfirstlane(blv.x),
                            __builtin_amdgcn_readfirstlane(blv.y));
  const int64_t kb0 = step_base(kbase, systems);
  const SysDesc& s = systems[bl.x];
  desc_prefetch(s);
  const int64_t k = kb0 + koff - s.k_origin;  // local step
  if (k < 0 || k >= s.total_steps) return;
  const int i = bl.y * 256 + threadIdx.x;
  const int cur = (int)(k & 1);
  double mx = 0.0;
  if (i < s.n) {
    const NPState st = np_state(s, i, cur);
    double fx, fy, fz;
    sum_parts(s, i, fx, fy, fz);  // partial sums of the source parts, fixed order
    mx = np_epilogue<kScan>(s, i, k, cur, fx, fy, fz, st);
  }
  if (k >= s.kept0 && !s.field_only) {  // the loop record: wave sums or their total
    double v = mx;
    v = wave_sum(v);
    double* rp = s.recpart + ((k - s.kept0) * s.ntiles + bl.y) * s.rec_slots;
    if (s.rec_slots == kRecSlots) {
      if ((threadIdx.x & 63) == 0) rp[threadIdx.x >> 6] = v;
    } else {  // uniform over the block
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
      __syncthreads();
      if (threadIdx.x == 0) rp[0] = (red[0] + red[1]) + (red[2] + red[3]);
    }
  }
}

// The special cases of k_update3 (field along or across the axis, K = 0, diagnostics)
// out of line: kept apart, the role paths schedule as a small kernel (measured: inlining
// it slowed the update of one N = 5000 assembly with three replicas from 11.9 to 12.3 us).
__device__ __noinline__ double np_epilogue_rare(const SysDesc& s, int i, int64_t k, int cur,
                                                double ax, double ay, double az) {
  return np_epilogue<false>(s, i, k, cur, ax, ay, az);
}

// Launches of at most kUpdate3MaxBlocks 256-particle blocks use k_update3; every system
// in them keeps one loop-record slot per wave (rec_slots_for).

// Per-particle update with the roots of the fall spread over three waves per particle
// (exact extremum search). Each 256-particle update block runs as four sub-blocks of 64
// particles and three waves: role 0 finds the global minimum, role 1 t* and the saddle,
// role 2 t* and the metastable minimum, for the same particles; the roles meet in LDS
// and role 0 finishes steps v-vii and writes the outputs and its wave's loop-record
// slot. On a launch with fewer waves than SIMDs the three chains run side by side, so a
// step waits for the longest of them instead of their sum, and small sub-blocks spread
// the chains over four times as many CUs, so fewer of them share a SIMD's issue. Each
// piece is the one sw_fall runs, so the results are those of k_update.
// Special cases (field along or across the axis, K = 0, diagnostics) run whole on role 0.
__global__ __launch_bounds__(192) void k_update3(const SysDesc* __restrict__ systems,
                                                 const int2* __restrict__ blocks,
                                                 const int64_t* __restrict__ kbase,
                                                 int64_t koff) {
  __shared__ double2 sh_r2a[64], sh_r2b[64];
  __shared__ int sh_two[64];
  // the sub-block's (system, particle block) is uniform: keep it in scalar registers, so
  // the descriptor is read with scalar loads and data loads are not chained behind it
  const int2 blv = blocks[blockIdx.x >> 2];
  const int2 bl = make_int2(__builtin_amdgcn_readfirstlane(blv.x),
                            __builtin_amdgcn_readfirstlane(blv.y));
  const int part = (int)(blockIdx.x & 3);  // sub-block = wave of the 256-particle block
  const int64_t kb0 = step_base(kbase, systems);
  const SysDesc& s = systems[bl.x];
  desc_prefetch(s);
  const int64_t k = kb0 + koff - s.k_origin;  // local step
  if (k < 0 || k >= s.total_steps) return;                      // uniform over the block
  const int role = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int i = bl.y * 256 + part * 64 + t;
  const int cur = (int)(k & 1);
  const bool act = i < s.n;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  bool general = false;
  NPIn q;
  Plane w;
  SWArgs a;
  Dir d1{0.0, 0.0};
  double u = 0.0;
  if (act) {
    const NPState st = np_state(s, i, cur);
    sum_parts(s, i, fx, fy, fz);  // partial sums of the source parts, fixed order
    if (!s.field_only && s.np.aniso) {
      q = np_in(s, k, fx, fy, fz, st.mo, st.nn);
      w = working_plane(s.np, q.Bx, q.By, q.Bz, q.nn.x, q.nn.y, q.nn.z, q.mo.x, q.mo.y, q.mo.z);
      general = w.hy != 0.0 && w.hx != 0.0;
    }
    if (general) {
      a = sw_args(w.hx, w.hy);
      if (role == 0) {
        d1 = sw_min1(a);
        // the step's uniform number, drawn while roles 1 and 2 find their roots
        if (s.np.thermal) u = philox_uniform(s.seed, s.stream, i, k);
      } else {
        const SWT tt = sw_tstar(a);
        if (role == 1) {
          sh_two[t] = tt.two ? 1 : 0;
          if (tt.two) {
            const Dir d = sw_saddle(a, tt);
            sh_r2a[t] = make_double2(d.s, d.c);
          }
        } else if (tt.two) {
          const Dir d = sw_meta(a, tt);
          sh_r2b[t] = make_double2(d.s, d.c);
        }
      }
    }
  }
  __syncthreads();
  double mx = 0.0;
  if (role == 0 && act) {
    if (general) {
      np_dhdip(s, i, k, fx, fy, fz);
      const bool two = sh_two[t] != 0;
      const Dir d2a = two ? Dir{sh_r2a[t].x, sh_r2a[t].y} : Dir{0.0, 0.0};
      const Dir d2b = two ? Dir{sh_r2b[t].x, sh_r2b[t].y} : Dir{0.0, 0.0};
      const SWState sw = sw_finish(a, w.d0, d1, two, d2a, d2b);
      const NPResult r =
          np_finish_with(s.np, w, sw, q.nn.x, q.nn.y, q.nn.z, [&] { return u; });
      mx = np_out(s, i, k, cur, q, r);
    } else {
      mx = np_epilogue_rare(s, i, k, cur, fx, fy, fz);
    }
  }
  if (role == 0 && k >= s.kept0 && !s.field_only) {  // uniform over the wave
    double v = mx;
    v = wave_sum(v);
    if (t == 0) s.recpart[((k - s.kept0) * s.ntiles + bl.y) * kRecSlots + part] = v;
    // (rec_slots == kRecSlots here: the launch holds at most kUpdate3MaxBlocks blocks)
  }
}

// ---------------------------------------------------------------------------
// End of run: per-system loop record and area, per-assembly replica statistics.
// ---------------------------------------------------------------------------
// out_sys[sys] = loop area (J/m^3, mean over particles and kept periods);
// rec_out rows: sum over tiles of the partial m_x sums (fixed order).
__global__ __launch_bounds__(256) void k_finalize_sys(const SysDesc* __restrict__ systems) {
  __shared__ double red[4];
  const SysDesc s = systems[blockIdx.x];
  const int tid = threadIdx.x;
  double a = 0.0;
  for (int i = tid; i < s.n; i += 256) a += s.area[i] + s.area[s.n + i];
  const double tot = block_sum_256(a, red);
  const int nk = (s.total_steps - s.kept0) / s.S;
  if (tid == 0) s.sys_area[0] = nk > 0 ? tot / ((double)s.n * nk) : 0.0;
  double* ro = s.rec;
  const int rows = s.total_steps - s.kept0;
  for (int r = tid; r < rows; r += 256) {
    double v = 0.0;
    for (int q = 0; q < s.ntiles; ++q) {
      const double* w = s.recpart + ((int64_t)r * s.ntiles + q) * s.rec_slots;
      v += s.rec_slots == kRecSlots ? (w[0] + w[1]) + (w[2] + w[3]) : w[0];
    }
    ro[r] = v;
  }
}

// Replica statistics of one assembly: mean and standard error of the per-replica
// areas (ddof = 1), single block.
__global__ __launch_bounds__(256) void k_finalize_asm(const double* __restrict__ sys_area, int R,
                                                      double* __restrict__ out) {
  __shared__ double red[4];
  double a = 0.0;
  for (int r = threadIdx.x; r < R; r += 256) a += sys_area[r];
  const double mean = block_sum_256(a, red) / R;
  double v = 0.0;
  for (int r = threadIdx.x; r < R; r += 256) {
    const double d = sys_area[r] - mean;
    v += d * d;
  }
  const double ss = block_sum_256(v, red);
  if (threadIdx.x == 0) {
    out[0] = mean;
    out[1] = R > 1 ? sqrt(ss / (R - 1) / R) : 0.0;
  }
}

// Replica-mean area of each particle (sum + compensation) / kept periods.
__global__ void k_area_per_np(const double* __restrict__ area, int n, int R, int n_kept,
                              double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = 0.0;
  for (int r = 0; r < R; ++r) a += area[(int64_t)r * 2 * n + i] + area[(int64_t)r * 2 * n + n + i];
  out[i] = n_kept > 0 ? a / ((double)R * n_kept) : 0.0;
}

// Deterministic mean-magnetisation loop of non-interacting particles (the paper's
// validation method, Sec. II.3 and Fig. 1(c)-(d)): one thread carries one particle of
// one replica through every step of the run. Its state is two weighted moments (wells A
// and B, all weight in A at the start); each step both fall in the applied field
// (steps iii-v), the weights are pooled by the minimum they reach, and Eq. 5 moves
// w_c P(c->o) from each well to the other (steps vi-vii); with one minimum all weight
// goes to it. The expected m_x feeds the loop record (fixed-order block sums per kept
// step) and the per-particle compensated area, as a kMC run does, so the same
// finalisation gives the loop, the area and the SAR. Requires K > 0 and no
// interactions (the launcher's caller checks both).
__global__ __launch_bounds__(256) void k_master(const SysDesc* __restrict__ systems) {
  __shared__ double red[4];
  const SysDesc& s = systems[blockIdx.y];
  if ((int)blockIdx.x * 256 >= s.n) return;  // whole block past this system's particles
  const int i = blockIdx.x * 256 + threadIdx.x;
  const bool act = i < s.n;
  const D4 nn = s.axes[act ? i : s.n - 1];  // idle lanes shadow the last particle
  const double ex = s.eh[0], ey = s.eh[1], ez = s.eh[2];
  MasterState q;
  master_init(q, nn.x, nn.y, nn.z, ex, ey, ez);
  double mx_prev = q.ax * ex + q.ay * ey + q.az * ez, sum = 0.0, comp = 0.0;
  for (int k = 0; k < s.total_steps; ++k) {
    const double Bext = applied_field(s, k);
    const double mx = master_step(s.np, Bext, ex, ey, ez, nn.x, nn.y, nn.z, q);
    if (k >= s.kept0) {
      neumaier_add(sum, comp, s.Ms * Bext * (mx - mx_prev));
      const double t = block_sum_256(act ? mx : 0.0, red);
      if ((int)threadIdx.x < s.rec_slots)
        s.recpart[((int64_t)(k - s.kept0) * s.ntiles + blockIdx.x) * s.rec_slots + threadIdx.x] =
            threadIdx.x == 0 ? t : 0.0;
    }
    mx_prev = mx;
  }
  if (act) {
    s.area[i] = sum;
    s.area[s.n + i] = comp;
    D4 m;  // expected moment after the last step, in the buffer that step writes
    m.x = q.wa * q.ax + q.wb * q.bx;
    m.y = q.wa * q.ay + q.wb * q.by;
    m.z = q.wa * q.az + q.wb * q.bz;
    m.w = 0.0;
    s.m64[(int64_t)(s.total_steps & 1) * s.stride + i] = m;
  }
}

// Local volume concentration, Eq. 8: phi_N = N / (8 (r_N/d)^3) with r_N the distance
// to the N-th nearest other particle (positions in units of d). The N-th smallest
// squared distance is found exactly by bisection on its bit pattern (non-negative
// doubles order like their bits): 64 passes, each counting the squared distances at
// or below the candidate over positions staged through LDS, keep the smallest value
// with at least N of them. Squared distances are dx*dx + dy*dy + dz*dz.
__global__ __launch_bounds__(256) void k_local_conc(const D4* __restrict__ pos, int n, int N,
                                                    double* __restrict__ phi) {
  __shared__ double sx[1024], sy[1024], sz[1024];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const D4 pi = pos[i < n ? i : n - 1];
  uint64_t lo = 0, hi = 0x7FF0000000000000ull;  // +0 .. +inf
  for (int pass = 0; pass < 64; ++pass) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    const double t = __longlong_as_double((long long)mid);
    int cnt = 0;
    for (int c0 = 0; c0 < n; c0 += 1024) {
      const int cn = min(1024, n - c0);
      __syncthreads();
      for (int j = threadIdx.x; j < cn; j += 256) {
        const D4 p = pos[c0 + j];
        sx[j] = p.x;
        sy[j] = p.y;
        sz[j] = p.z;
      }
      __syncthreads();
      for (int j = 0; j < cn; ++j) {
        const double dx = sx[j] - pi.x, dy = sy[j] - pi.y, dz = sz[j] - pi.z;
        const double d2 = dx * dx + dy * dy + dz * dz;
        cnt += (c0 + j != i && d2 <= t) ? 1 : 0;
      }
    }
    if (lo < hi) {
      if (cnt >= N)
        hi = mid;
      else
        lo = mid + 1;
    }
  }
  if (i < n) {
    const double r = sqrt(__longlong_as_double((long long)lo));
    phi[i] = (double)N / (8.0 * r * r * r);
  }
}

// Start of a run: m_i = sign(n_i . x) n_i in buffer 0 (both precisions), zero the
// area accumulators and the loop-record partials.
__global__ void k_init(const SysDesc* __restrict__ systems) {
  const SysDesc s = systems[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < s.n) {
    const D4 a = s.axes[i];
    const double sg = a.x * s.eh[0] + a.y * s.eh[1] + a.z * s.eh[2] >= 0.0 ? 1.0 : -1.0;
    D4 m;
    m.x = sg * a.x;
    m.y = sg * a.y;
    m.z = sg * a.z;
    m.w = 0.0;
    s.m64[i] = m;
    if (s.m32) {
      F4 f;
      f.x = (float)m.x;
      f.y = (float)m.y;
      f.z = (float)m.z;
      f.w = 0.f;
      s.m32[i] = f;
    }
    s.area[i] = 0.0;
    s.area[s.n + i] = 0.0;
    if (s.dhdip) s.dhdip[i] = 0.0;
  }
  const int64_t rows = (int64_t)(s.total_steps - s.kept0) * s.ntiles * s.rec_slots;
  for (int64_t r = i; r < rows; r += (int64_t)gridDim.x * blockDim.x) s.recpart[r] = 0.0;
}

// Copy FP64 moments of buffer b into the FP32 field copy.
__global__ void k_sync32(const SysDesc* __restrict__ systems, int b) {
  const SysDesc s = systems[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n || !s.m32) return;
  const D4 m = s.m64[(int64_t)b * s.stride + i];
  F4 f;
  f.x = (float)m.x;
  f.y = (float)m.y;
  f.z = (float)m.z;
  f.w = 0.f;
  s.m32[(int64_t)b * s.stride + i] = f;
}

// ---------------------------------------------------------------------------
// Diagnostics for unit parity
// ---------------------------------------------------------------------------
__global__ void k_philox_raw(uint64_t seed, uint64_t stream, const uint64_t* __restrict__ ctr,
                             uint64_t* __restrict__ out, int64_t nblk) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  uint64_t c0 = ctr[4 * b], c1 = ctr[4 * b + 1], c2 = ctr[4 * b + 2], c3 = ctr[4 * b + 3];
  philox4x64_10(c0, c1, c2, c3, seed, stream);
  out[4 * b] = c0;
  out[4 * b + 1] = c1;
  out[4 * b + 2] = c2;
  out[4 * b + 3] = c3;
}

__global__ void k_sw(const double* __restrict__ hx, const double* __restrict__ hy,
                     const double* __restrict__ th0, double* __restrict__ out, int64_t n,
                     int scan200) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Dir d;
  sincos(th0[i], &d.s, &d.c);
  const SWState r = scan200 ? sw_fall_scan200(hx[i], hy[i], d) : sw_fall(hx[i], hy[i], d);
  double* o = out + 6 * i;
  o[0] = atan2(r.s_c, r.c_c);
  o[1] = r.e_c;
  o[2] = atan2(r.s_o, r.c_o);
  o[3] = r.e_o;
  o[4] = r.e3;
  o[5] = r.two ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
// Plan of one Eq. 1 field evaluation in caller-provided device memory: the descriptor
// (passed by value), the part-major field tile list and the update block list of the
// single system, and the caller's moments (n x 3 doubles) as the buffer-0 moments of
// the descriptor (FP64, and the FP32 copy when m32 is set). Written by kernels, so
// the plan needs neither a host copy nor an allocation.
// ---------------------------------------------------------------------------
__global__ void k_field_plan(SysDesc s, SysDesc* __restrict__ d_desc, int4* __restrict__ tiles,
                             int tiles_per_part, int nsplit, int2* __restrict__ ublocks,
                             int nublocks, const double* __restrict__ m_in) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *d_desc = s;
  if (i < tiles_per_part * nsplit) tiles[i] = make_int4(0, i % tiles_per_part, 1, i / tiles_per_part);
  if (i < nublocks) ublocks[i] = make_int2(0, i);
  if (i < s.n) {
    D4 m;
    m.x = m_in[3 * i];
    m.y = m_in[3 * i + 1];
    m.z = m_in[3 * i + 2];
    m.w = 0.0;
    s.m64[i] = m;
    if (s.m32) {
      F4 f;
      f.x = (float)m.x;
      f.y = (float)m.y;
      f.z = (float)m.z;
      f.w = 0.f;
      s.m32[i] = f;
    }
  }
}

// The three field components of each particle's diagnostics record (8 doubles) into
// an n x 3 array.
__global__ void k_field_out(const double* __restrict__ diag, double* __restrict__ B, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  B[3 * i] = diag[8 * i];
  B[3 * i + 1] = diag[8 * i + 1];
  B[3 * i + 2] = diag[8 * i + 2];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t launch_resident(bool fp64, bool scan, const SysDesc* d_sys, int nsys, int64_t k0,
                           int64_t k1, int nmax, hipStream_t st) {
  if (nsys == 0) return hipSuccess;
  if (fp64) {
    const size_t lds = (size_t)nmax * 3 * sizeof(D4);
    if (scan)
      hipLaunchKernelGGL((k_resident<double, true>), dim3(nsys), dim3(kResThreads), lds, st, d_sys, k0, k1,
                         nmax);
    else
      hipLaunchKernelGGL((k_resident<double, false>), dim3(nsys), dim3(kResThreads), lds, st, d_sys, k0,
                         k1, nmax);
  } else {
    const size_t lds = (size_t)nmax * 3 * sizeof(F4);
    if (scan)
      hipLaunchKernelGGL((k_resident<float, true>), dim3(nsys), dim3(kResThreads), lds, st, d_sys, k0, k1,
                         nmax);
    else
      hipLaunchKernelGGL((k_resident<float, false>), dim3(nsys), dim3(kResThreads), lds, st, d_sys, k0, k1,
                         nmax);
  }
  return hipGetLastError();
}

size_t resident_lds_bytes(bool fp64, int nmax) {
  return fp64 ? (size_t)nmax * 3 * sizeof(D4) : (size_t)nmax * 3 * sizeof(F4);
}

hipError_t set_resident_lds_limit() {
  const void* fns[] = {(const void*)k_resident<double, false>, (const void*)k_resident<float, false>,
                       (const void*)k_resident<double, true>, (const void*)k_resident<float, true>};
  for (const void* f : fns) {
    // the whole 160 KB of a CU's LDS less the kernel's static arrays
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, f);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024 - (int)attr.sharedSizeBytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int tile_width(int kind) { return kind == 0 ? 64 : 16; }

// kind 0: 64 targets per field block, kind 1: 16 targets per field block; G replicas
// of one assembly share each block (FP32 only for G > 1)
template <typename T, int TI>
static void launch_field_g(int G, const SysDesc* d_sys, const int4* d_tiles, int ntiles,
                           const int64_t* kbase, int64_t koff, hipStream_t st) {
  switch (G) {
    case 4:
      hipLaunchKernelGGL((k_field<T, TI, 4>), dim3(ntiles), dim3(1024), 0, st, d_sys, d_tiles, kbase, koff);
      break;
    case 3:
      hipLaunchKernelGGL((k_field<T, TI, 3>), dim3(ntiles), dim3(1024), 0, st, d_sys, d_tiles, kbase, koff);
      break;
    case 2:
      hipLaunchKernelGGL((k_field<T, TI, 2>), dim3(ntiles), dim3(1024), 0, st, d_sys, d_tiles, kbase, koff);
      break;
    default:
      hipLaunchKernelGGL((k_field<T, TI, 1>), dim3(ntiles), dim3(1024), 0, st, d_sys, d_tiles, kbase, koff);
  }
}

hipError_t launch_field(bool fp64, int kind, int G, const SysDesc* d_sys, const int4* d_tiles,
                        int ntiles, const int64_t* kbase, int64_t koff, hipStream_t st) {
  if (ntiles == 0) return hipSuccess;
  if (fp64) {
    if (kind == 0)
      hipLaunchKernelGGL((k_field<double, 64, 1>), dim3(ntiles), dim3(1024), 0, st, d_sys, d_tiles,
                         kbase, koff);
    else
      hipLaunchKernelGGL((k_field<double, 16, 1>), dim3(ntiles), dim3(1024), 0, st, d_sys, d_tiles,
                         kbase, koff);
  } else {
    if (kind == 0)
      launch_field_g<float, 64>(G, d_sys, d_tiles, ntiles, kbase, koff, st);
    else
      launch_field_g<float, 16>(G, d_sys, d_tiles, ntiles, kbase, koff, st);
  }
  return hipGetLastError();
}

hipError_t launch_update(bool scan, const SysDesc* d_sys, const int2* d_blocks, int nblocks,
                         const int64_t* kbase, int64_t koff, hipStream_t st) {
  if (nblocks == 0) return hipSuccess;
  // the three-role form pays while the blocks leave CUs idle; beyond that its duplicated
  // work (plane and t* on three and two waves) costs more than the shorter chains save.
  // Both forms compute the same pieces in the same order, so the choice does not change
  // results (tested across the threshold)
  if (scan)
    hipLaunchKernelGGL(k_update<true>, dim3(nblocks), dim3(256), 0, st, d_sys, d_blocks, kbase,
                       koff);
  else if (nblocks <= kUpdate3MaxBlocks)
    hipLaunchKernelGGL(k_update3, dim3(4 * nblocks), dim3(192), 0, st, d_sys, d_blocks, kbase,
                       koff);
  else
    hipLaunchKernelGGL(k_update<false>, dim3(nblocks), dim3(256), 0, st, d_sys, d_blocks, kbase,
                       koff);
  return hipGetLastError();
}

hipError_t launch_field_plan(const SysDesc& s, SysDesc* d_desc, int4* tiles, int tiles_per_part,
                             int nsplit, int2* ublocks, int nublocks, const double* m_in,
                             hipStream_t st) {
  const int cnt = max(max(s.n, tiles_per_part * nsplit), max(nublocks, 1));
  hipLaunchKernelGGL(k_field_plan, dim3((cnt + 255) / 256), dim3(256), 0, st, s, d_desc, tiles,
                     tiles_per_part, nsplit, ublocks, nublocks, m_in);
  return hipGetLastError();
}

hipError_t launch_empty_steps(int64_t steps, double* sink, hipStream_t st) {
  hipLaunchKernelGGL(k_empty_steps, dim3(1), dim3(kResThreads), 0, st, steps, sink);
  return hipGetLastError();
}

hipError_t launch_field_out(const double* diag, double* B, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_field_out, dim3((n + 255) / 256), dim3(256), 0, st, diag, B, n);
  return hipGetLastError();
}

__global__ void k_set_step(int64_t* kbase, int64_t v, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *kbase = add ? *kbase + v : v;
}

hipError_t launch_set_step(int64_t* kbase, int64_t v, bool add, hipStream_t st) {
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, st, kbase, v, add ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_finalize(const SysDesc* d_sys, int nsys, hipStream_t st) {
  if (nsys == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize_sys, dim3(nsys), dim3(256), 0, st, d_sys);
  return hipGetLastError();
}

hipError_t launch_local_conc(const D4* pos, int n, int N, double* phi, hipStream_t st) {
  hipLaunchKernelGGL(k_local_conc, dim3((n + 255) / 256), dim3(256), 0, st, pos, n, N, phi);
  return hipGetLastError();
}

hipError_t launch_master(const SysDesc* d_sys, int nsys, int nmax, hipStream_t st) {
  if (nsys == 0) return hipSuccess;
  hipLaunchKernelGGL(k_master, dim3((nmax + 255) / 256, nsys), dim3(256), 0, st, d_sys);
  return hipGetLastError();
}

hipError_t launch_init(const SysDesc* d_sys, int nsys, int nmax, hipStream_t st) {
  if (nsys == 0) return hipSuccess;
  hipLaunchKernelGGL(k_init, dim3((nmax + 255) / 256, nsys), dim3(256), 0, st, d_sys);
  return hipGetLastError();
}

hipError_t launch_sync32(const SysDesc* d_sys, int nsys, int nmax, int b, hipStream_t st) {
  if (nsys == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sync32, dim3((nmax + 255) / 256, nsys), dim3(256), 0, st, d_sys, b);
  return hipGetLastError();
}

hipError_t launch_finalize_asm(const double* d_sys_area, int R, double* d_out, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_asm, dim3(1), dim3(256), 0, st, d_sys_area, R, d_out);
  return hipGetLastError();
}

hipError_t launch_area_per_np(const double* d_area, int n, int R, int n_kept, double* d_out,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_area_per_np, dim3((n + 255) / 256), dim3(256), 0, st, d_area, n, R, n_kept,
                     d_out);
  return hipGetLastError();
}

hipError_t launch_philox_raw(uint64_t seed, uint64_t stream, const uint64_t* d_ctr, uint64_t* d_out,
                             int64_t nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_philox_raw, dim3((unsigned)((nblk + 255) / 256)), dim3(256), 0, st, seed,
                     stream, d_ctr, d_out, nblk);
  return hipGetLastError();
}

hipError_t launch_sw(const double* hx, const double* hy, const double* th0, double* out, int64_t n,
                     bool scan200, hipStream_t st) {
  hipLaunchKernelGGL(k_sw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, hx, hy, th0, out,
                     n, scan200 ? 1 : 0);
  return hipGetLastError();
}

}  // namespace mh
