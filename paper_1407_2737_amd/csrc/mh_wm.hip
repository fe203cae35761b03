// Replica-batched interaction-matrix form of Eq. 1 on MFMA (gfx950).
//
// The positions of an assembly are fixed during a run, so the dipolar field of Eq. 1
// is a fixed linear map of the moments: B = C W m with W (3N x 3N) made of the 3x3
// blocks T_ij = (3 e_ij e_ij^T - I) / r_ij^3 (zero for i = j), in units of d. Applied
// to the moments of R independent replicas at once it is a dense product W M with
// M (3N x R) the moments of all replicas.
//
// Precision: W and M are split into BF16 hi + lo parts (hi = bf16(x),
// lo = bf16(x - hi)); W M ~ W_hi M_hi + W_hi M_lo + W_lo M_hi with FP32 accumulation
// on v_mfma_f32_32x32x16_bf16. The kernel computes B^T = M^T W^T: the A operand is
// rows of M^T (one replica, k contiguous) and the B operand is rows of W (k
// contiguous), and it writes B^T (replica-major), which the per-particle update then
// reads contiguously.
//
// W is never stored: each block generates its W tile stage by stage from the
// positions (FP64 differences, FP32 r^-3 and r^-5 terms, then the hi/lo split), so
// the only operand streamed from memory is M^T. Generation costs about a quarter of
// the block's MFMA time in VALU work, issued between the wave's own MFMAs.
//
// Tiling: block = 8 waves, tile = 256 replicas x 192 matrix rows (64 target particles)
// over half of k (two k splits whose partial products the update kernel adds in fixed
// order), k-stage 48 (16 source particles). Thread (tp, c) = (tid / 8, tid % 8)
// generates the 3x3 blocks of target tp with sources 2c and 2c + 1 of the next stage
// (rows 3 tp .. 3 tp + 2, columns 6 c .. 6 c + 5) into the other LDS buffer (hi and
// lo, rows padded to 56 bf16 so that 16-byte fragment reads do not conflict), a third
// per k-step, its VALU work interleaved with that k-step's MFMAs (two VALU per MFMA);
// the stage's 16 source positions are staged in LDS one stage earlier. Each wave owns
// 32 replicas x 192 rows (six 32x32 accumulators) and loads its M^T fragments straight
// from global memory, each k-step's fragment one stage ahead. An XCD (block index mod
// 8) works on one (k split, replica tile) pair where the shape allows it, so its
// blocks share one M^T slab in its L2.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mh_kernels.hpp"

namespace mh {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int WM_BM = 256;  // replicas per block
constexpr int WM_BN = 192;  // W rows per block (64 target particles)
constexpr int WM_BK = 48;   // k per stage (16 source particles)
constexpr int WM_SK = 2;    // k splits (partial products summed by the update)
constexpr int WM_LD = WM_BK + 8;
constexpr int WM_SUB = WM_BK / 16;  // MFMA k-steps per stage

__device__ __forceinline__ __bf16 bf16_rn(float x) { return (__bf16)x; }

// M^T is stored fragment-major: for replica tile r/32 and k-stage k/48, the 32 x 48
// block is laid out as [sub][lane][8] with lane = 32 * (kk / 24) + r % 32,
// sub = (kk % 24) / 8 (kk = k % 48), so the fragment load of one k-step by a wave is
// one contiguous 1 KB read.
__device__ __forceinline__ size_t mt_offset(int r, int k, int Kp) {
  const int rt = r >> 5, rr = r & 31;
  const int kb = k / WM_BK, kk = k - kb * WM_BK;
  const int lane = (kk / 24) * 32 + rr;
  const int sub = (kk % 24) >> 3;
  return ((((size_t)rt * (Kp / WM_BK) + kb) * WM_SUB + sub) * 64 + lane) * 8 + (kk & 7);
}

// bf16 hi/lo split of two values, packed with a in the low half (the lower address):
// one pair conversion (round to nearest even) for each part.
__device__ __forceinline__ void split_pack(float a, float b, uint32_t& hi, uint32_t& lo) {
  const f32x2 v = {a, b};
  const bf16x2 h = __builtin_convertvector(v, bf16x2);
  const bf16x2 l = __builtin_convertvector(v - __builtin_convertvector(h, f32x2), bf16x2);
  hi = __builtin_bit_cast(uint32_t, h);
  lo = __builtin_bit_cast(uint32_t, l);
}

// The 3x3 block T_ij (reduced units) of target position p and source q: q.w = 0 marks
// a missing source (padding), own = the target itself. Row a of the block in t[3a..];
// the block is symmetric, so its six distinct entries are computed once.
__device__ __forceinline__ void pair_block(double px, double py, double pz, bool tgt_ok,
                                           const D4& q, bool own, float* t) {
  const bool ok = tgt_ok && q.w != 0.0 && !own;
  const float dx = (float)(q.x - px), dy = (float)(q.y - py), dz = (float)(q.z - pz);
  const float r2 = ok ? dx * dx + dy * dy + dz * dz : 1.0f;
  const float inv = __builtin_amdgcn_rsqf(r2);
  const float inv2 = inv * inv;
  const float c3 = ok ? inv * inv2 : 0.0f;
  const float s5 = 3.0f * c3 * inv2;
  const float ux = dx * s5, uy = dy * s5, uz = dz * s5;
  t[0] = dx * ux - c3;
  t[1] = t[3] = dx * uy;
  t[2] = t[6] = dx * uz;
  t[4] = dy * uy - c3;
  t[5] = t[7] = dy * uz;
  t[8] = dz * uz - c3;
}

typedef __bf16 WTile[2][2][WM_BN][WM_LD];  // generated W tiles [buffer][hi/lo][row][k]
typedef D4 PStage[2][16];                     // source positions of two stages

// Block bid of the product of g, whose blocks are numbered 0 .. nb_range - 1 in a range
// of the launch that starts at a multiple of 8 (bid mod 8 is then the block's XCD).
__device__ __forceinline__ void wm_gemm_block(const WMArgs& g, int bid, int nb_range, WTile& Ws,
                                              PStage& Ps) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  // block -> (W row tile, k split, replica tile). XCD-aware when the shape allows it:
  // the C = n_ctiles * WM_SK (k split, replica tile) pairs each get 8 / C XCDs, so the
  // blocks of an XCD read one M^T slab, from that XCD's L2
  int rt, ks, ct;
  const unsigned ub = (unsigned)bid;
  const int nb = g.n_rtiles * g.n_ctiles * WM_SK;
  const int C = g.n_ctiles * WM_SK;
  if ((C == 1 || C == 2 || C == 4 || C == 8) && nb == nb_range && g.n_rtiles % (8 / C) == 0) {
    const int X = 8 / C;  // XCDs per pair
    const int xcd = ub & 7, slot = ub >> 3;
    const int pair = xcd / X;
    ks = pair % WM_SK;
    ct = pair / WM_SK;
    rt = (xcd % X) * (g.n_rtiles / X) + slot;
  } else {
    ct = ub % g.n_ctiles;
    ks = (ub / g.n_ctiles) % WM_SK;
    rt = ub / (g.n_ctiles * WM_SK);
  }
  const int wrow0 = rt * WM_BN;           // first W row (output column) of the block
  const int rep0 = ct * WM_BM + w * 32;   // the wave's 32 replicas (output rows)
  const int kbeg = ks * (g.Kp / WM_SK);
  const int jbeg = kbeg / 3;              // first source particle of the k split
  const int nst = g.Kp / WM_SK / WM_BK;
  // M^T fragments of the wave's 32-replica tile (fragment-major layout, see mt_offset)
  const int nkb = g.Kp / WM_BK;
  const size_t aoff = (size_t)(rep0 >> 5) * nkb * WM_SUB * 512 + (size_t)lane * 8;
  const __bf16* ah = g.mhi + aoff;
  const __bf16* al = g.mlo + aoff;
  // M^T fragments of the stage's k-steps [hi/lo][k-step]: slot s is reloaded with k-step s
  // of the next stage as soon as the MFMAs of k-step s are issued
  bf16x8 ac[2][WM_SUB];
  auto load_a = [&](int st_, int s) {
    const size_t o = (size_t)(kbeg / WM_BK + st_) * (WM_SUB * 512) + (size_t)s * 512;
    ac[0][s] = *reinterpret_cast<const bf16x8*>(ah + o);
    ac[1][s] = *reinterpret_cast<const bf16x8*>(al + o);
  };
  // generation: target tp of the block, sources 2c, 2c+1 of a stage
  const int tp = tid >> 3, c = tid & 7;
  const int it = rt * 64 + tp;
  const bool tgt_ok = it < g.n;
  const D4 pt = g.pos[tgt_ok ? it : 0];
  // source positions of stage st_ for threads 0..15: q.w = 1 marks a real particle
  auto src_of = [&](int st_) -> D4 {
    const int j = jbeg + 16 * st_ + tid;
    D4 q = {0.0, 0.0, 0.0, 0.0};
    if (st_ < nst && j < g.n) {
      q = g.pos[j];
      q.w = 1.0;
    }
    return q;
  };
  uint32_t gh[9], gl[9];  // generated rows 3tp..3tp+2 x columns 6c..6c+5, hi and lo
  auto generate = [&](int st_) {
    const int pb = st_ & 1;
    const int j0 = jbeg + 16 * st_ + 2 * c;
    float t0[9], t1[9];
    pair_block(pt.x, pt.y, pt.z, tgt_ok, Ps[pb][2 * c], j0 == it, t0);
    pair_block(pt.x, pt.y, pt.z, tgt_ok, Ps[pb][2 * c + 1], j0 + 1 == it, t1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      split_pack(t0[3 * a], t0[3 * a + 1], gh[3 * a], gl[3 * a]);
      split_pack(t0[3 * a + 2], t1[3 * a], gh[3 * a + 1], gl[3 * a + 1]);
      split_pack(t1[3 * a + 1], t1[3 * a + 2], gh[3 * a + 2], gl[3 * a + 2]);
    }
  };
  auto store_w = [&](int buf) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      uint32_t* dh = reinterpret_cast<uint32_t*>(&Ws[buf][0][3 * tp + a][6 * c]);
      uint32_t* dl = reinterpret_cast<uint32_t*>(&Ws[buf][1][3 * tp + a][6 * c]);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        dh[q] = gh[3 * a + q];
        dl[q] = gl[3 * a + q];
      }
    }
  };

  f32x16 acc[6];
#pragma unroll
  for (int u = 0; u < 6; ++u)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[u][e] = 0.f;

  // prologue: source positions of stages 0 and 1, W of stage 0, M^T of stage 0
#pragma unroll
  for (int s = 0; s < WM_SUB; ++s) load_a(0, s);
  if (tid < 16) {
    Ps[0][tid] = src_of(0);
    Ps[1][tid] = src_of(1);
  }
  __syncthreads();
  generate(0);
  store_w(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    const bool more = st + 1 < nst;
    D4 pnext = {0.0, 0.0, 0.0, 0.0};
    if (more && tid < 16) pnext = src_of(st + 2);
    // keep the next stage's loads in flight across the MFMAs
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    float t0[9], t1[9];
    const int j0 = jbeg + 16 * (st + 1) + 2 * c;
    const int pbn = (st + 1) & 1;
#pragma unroll
    for (int s = 0; s < WM_SUB; ++s) {
      const int kk = (lane >> 5) * 24 + s * 8;
      bf16x8 bh[6], bl[6];
#pragma unroll
      for (int u = 0; u < 6; ++u) {
        bh[u] = *reinterpret_cast<const bf16x8*>(&Ws[cur][0][u * 32 + (lane & 31)][kk]);
        bl[u] = *reinterpret_cast<const bf16x8*>(&Ws[cur][1][u * 32 + (lane & 31)][kk]);
      }
#pragma unroll
      for (int u = 0; u < 6; ++u)
        acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ac[0][s], bh[u], acc[u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < 6; ++u)
        acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ac[1][s], bh[u], acc[u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < 6; ++u)
        acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ac[0][s], bl[u], acc[u], 0, 0, 0);
      // a third of the next stage's W per k-step, between this k-step's MFMAs (also in
      // the last stage, where the sources are padding and nothing reads the result)
      if (s == 0) pair_block(pt.x, pt.y, pt.z, tgt_ok, Ps[pbn][2 * c], j0 == it, t0);
      if (s == 1) pair_block(pt.x, pt.y, pt.z, tgt_ok, Ps[pbn][2 * c + 1], j0 + 1 == it, t1);
      if (s == 2) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          split_pack(t0[3 * a], t0[3 * a + 1], gh[3 * a], gl[3 * a]);
          split_pack(t0[3 * a + 2], t1[3 * a], gh[3 * a + 1], gl[3 * a + 1]);
          split_pack(t1[3 * a + 1], t1[3 * a + 2], gh[3 * a + 2], gl[3 * a + 2]);
        }
        store_w(cur ^ 1);  // free: every wave finished reading it before the last barrier
      }
      if (more) load_a(st + 1, s);
      __builtin_amdgcn_sched_group_barrier(0x100, 12, 0);  // the k-step's LDS reads first
#pragma unroll
      for (int q = 0; q < 18; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // then up to 2 VALU
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    if (more) {
      // Ps[st & 1] (read for W of stage st + 1 above) takes the sources of stage st + 2
      if (tid < 16) Ps[st & 1][tid] = pnext;
      __syncthreads();
    }
  }
  // partial B^T of k split ks: lane holds column wrow0 + u*32 + lane%32 of rows
  // rep0 + 8*(e/4) + 4*(lane/32) + e%4
  float* bt = g.bt + (size_t)ks * g.Rp * g.Mp;
#pragma unroll
  for (int u = 0; u < 6; ++u)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int row = rep0 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
      const int col = wrow0 + u * 32 + (lane & 31);
      bt[(size_t)row * g.Mp + col] = acc[u][e];
    }
}

__global__ __launch_bounds__(512) void k_wm_gemm(WMArgs g) {
  __shared__ __attribute__((aligned(16))) WTile Ws;
  __shared__ PStage Ps;
  wm_gemm_block(g, blockIdx.x, gridDim.x, Ws, Ps);
}

// Item of a launch that covers several systems' products or matrix-form updates: the
// items own consecutive block ranges, in the order the host chose.
__device__ __forceinline__ int wm_item_of(const WMGroupItem* __restrict__ items, int nitems) {
  int q = 0;
  while (q + 1 < nitems && (int)blockIdx.x >= items[q + 1].boff) ++q;
  return q;
}

// The products of several systems in one launch (block ranges start at multiples of 8,
// so each block keeps the XCD it has in a launch of its own and computes the same tile).
__global__ __launch_bounds__(512) void k_wm_gemm_group(const WMGroupItem* __restrict__ items,
                                                       int nitems) {
  __shared__ __attribute__((aligned(16))) WTile Ws;
  __shared__ PStage Ps;
  const int q = wm_item_of(items, nitems);
  const int bid = (int)blockIdx.x - items[q].boff;
  if (bid >= items[q].nb) return;
  const WMArgs g = items[q].g;
  wm_gemm_block(g, bid, items[q].nb, Ws, Ps);
}

// hi/lo split of the moments of replica r, particle i into M^T.
__device__ __forceinline__ void store_split(const WMArgs& g, int r, int i, double mx, double my,
                                            double mz) {
  const double m[3] = {mx, my, mz};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const __bf16 h = bf16_rn((float)m[c]);
    const __bf16 l = bf16_rn((float)(m[c] - (double)(float)h));
    const size_t o = mt_offset(r, 3 * i + c, g.Kp);
    g.mhi[o] = h;
    g.mlo[o] = l;
  }
}

// Moments of buffer b of every replica into M^T (start of a run or after a host write).
__global__ void k_wm_pack(const SysDesc* __restrict__ systems, WMArgs g, int b) {
  const int r = blockIdx.y;
  const SysDesc& s = systems[r];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n) return;
  const D4 m = s.m64[(int64_t)b * s.stride + i];
  store_split(g, r, i, m.x, m.y, m.z);
}

// Per-particle update of the matrix form: thread (r, i) reads its three reduced field
// components from B^T, runs steps iii-vii and writes the new moment (FP64 state and the
// hi/lo split for the next product).
// Block (bx, r) covers particles 256 bx .. 256 bx + 255 of replica r.
template <bool kScan>
__device__ __forceinline__ void wm_update_block(const SysDesc* __restrict__ systems,
                                                const WMArgs& g, const int64_t* __restrict__ kbase,
                                                int64_t koff, int bx, int r, double* red) {
  const int64_t kb0 = step_base(kbase, systems);
  const SysDesc& s = systems[r];
  desc_prefetch(s);
  const int64_t k = kb0 + koff - s.k_origin;  // local step
  if (k < 0 || k >= s.total_steps) return;
  const int i = bx * 256 + threadIdx.x;
  const int cur = (int)(k & 1);
  double mx = 0.0;
  if (i < s.n) {
    const NPState st = np_state(s, i, cur);
    // partial products of the k splits, added in fixed order
    double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
    for (int q = 0; q < WM_SK; ++q) {
      const float* f = g.bt + (size_t)q * g.Rp * g.Mp + (size_t)r * g.Mp + 3 * i;
      fx += (double)f[0];
      fy += (double)f[1];
      fz += (double)f[2];
    }
    mx = np_epilogue<kScan>(s, i, k, cur, fx, fy, fz, st);
    if (!s.field_only) {
      const D4 m = s.m64[(int64_t)(cur ^ 1) * s.stride + i];
      store_split(g, r, i, m.x, m.y, m.z);
    }
  }
  if (k >= s.kept0 && !s.field_only) {
    double v = mx;
    v = wave_sum(v);
    double* rp = s.recpart + ((k - s.kept0) * s.ntiles + bx) * s.rec_slots;
    if (s.rec_slots == kRecSlots) {
      if ((threadIdx.x & 63) == 0) rp[threadIdx.x >> 6] = v;
    } else {  // uniform over the block
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
      __syncthreads();
      if (threadIdx.x == 0) rp[0] = (red[0] + red[1]) + (red[2] + red[3]);
    }
  }
}

template <bool kScan>
__global__ __launch_bounds__(256) void k_wm_update(const SysDesc* __restrict__ systems, WMArgs g,
                                                   const int64_t* __restrict__ kbase,
                                                   int64_t koff) {
  __shared__ double red[4];
  wm_update_block<kScan>(systems, g, kbase, koff, blockIdx.x, blockIdx.y, red);
}

// The matrix-form updates of several systems in one launch: item q owns nb = nbx x R
// blocks from boff on, block boff + r nbx + bx being (bx, r) of its own launch.
template <bool kScan>
__global__ __launch_bounds__(256) void k_wm_update_group(const SysDesc* __restrict__ all,
                                                         const WMGroupItem* __restrict__ items,
                                                         int nitems,
                                                         const int64_t* __restrict__ kbase,
                                                         int64_t koff) {
  __shared__ double red[4];
  const int q = wm_item_of(items, nitems);
  const int lb = (int)blockIdx.x - items[q].boff;
  if (lb >= items[q].nb) return;
  const int nbx = items[q].nbx;
  const WMArgs g = items[q].g;
  wm_update_block<kScan>(all + items[q].first, g, kbase, koff, lb % nbx, lb / nbx, red);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
int wm_tile_rows() { return WM_BN; }
int wm_tile_reps() { return WM_BM; }
int wm_tile_k() { return WM_BK * WM_SK; }
int wm_ksplit() { return WM_SK; }

hipError_t launch_wm_gemm(const WMArgs& g, hipStream_t st) {
  hipLaunchKernelGGL(k_wm_gemm, dim3(g.n_rtiles * g.n_ctiles * WM_SK), dim3(512), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_wm_update(bool scan, const SysDesc* d_sys, int R, int n, const WMArgs& g,
                            const int64_t* kbase, int64_t koff, hipStream_t st) {
  if (scan)
    hipLaunchKernelGGL(k_wm_update<true>, dim3((n + 255) / 256, R), dim3(256), 0, st, d_sys, g,
                       kbase, koff);
  else
    hipLaunchKernelGGL(k_wm_update<false>, dim3((n + 255) / 256, R), dim3(256), 0, st, d_sys, g,
                       kbase, koff);
  return hipGetLastError();
}

hipError_t launch_wm_gemm_group(const WMGroupItem* d_items, int nitems, int nblocks,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_wm_gemm_group, dim3(nblocks), dim3(512), 0, st, d_items, nitems);
  return hipGetLastError();
}

hipError_t launch_wm_update_group(bool scan, const SysDesc* d_all, const WMGroupItem* d_items,
                                  int nitems, int nblocks, const int64_t* kbase, int64_t koff,
                                  hipStream_t st) {
  if (scan)
    hipLaunchKernelGGL(k_wm_update_group<true>, dim3(nblocks), dim3(256), 0, st, d_all, d_items,
                       nitems, kbase, koff);
  else
    hipLaunchKernelGGL(k_wm_update_group<false>, dim3(nblocks), dim3(256), 0, st, d_all, d_items,
                       nitems, kbase, koff);
  return hipGetLastError();
}

hipError_t launch_wm_pack(const SysDesc* d_sys, int R, int n, const WMArgs& g, int b,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_wm_pack, dim3((n + 255) / 256, R), dim3(256), 0, st, d_sys, g, b);
  return hipGetLastError();
}

}  // namespace mh
