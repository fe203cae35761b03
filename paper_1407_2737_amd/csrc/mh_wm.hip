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
// Tiling: block = 8 waves, tile = 256 replicas x 192 matrix rows over half of k (two k
// splits whose partial products the update kernel adds in fixed order), k-stage 64.
// The 192 W rows of a stage (hi and lo) are staged through LDS (double buffered, rows
// padded to 72 bf16 so that 16-byte fragment reads do not conflict); each wave owns 32
// replicas x 192 rows (six 32x32 accumulators) and loads its M^T fragments straight
// from global memory, one stage ahead. The tile size sets the operand traffic from L2
// per step: W once per replica tile (2x), M^T once per W row tile (3N/192 x). An XCD
// (block index mod 8) owns whole W row tiles, so each W slab comes from HBM once.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mh_kernels.hpp"

namespace mh {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int WM_BM = 256;  // replicas per block
constexpr int WM_BN = 192;  // W rows per block
constexpr int WM_BK = 64;   // k per stage
constexpr int WM_SK = 2;    // k splits (partial products summed by the update)
constexpr int WM_LD = WM_BK + 8;

__device__ __forceinline__ __bf16 bf16_rn(float x) { return (__bf16)x; }

// M^T is stored fragment-major: for replica tile r/32 and k-stage k/64, the 32 x 64
// block is laid out as [sub][lane][8] with lane = 32 * (kk / 32) + r % 32,
// sub = (kk % 32) / 8 (kk = k % 64), so the fragment load of one substep by a wave is
// one contiguous 1 KB read.
__device__ __forceinline__ size_t mt_offset(int r, int k, int Kp) {
  const int rt = r >> 5, rr = r & 31;
  const int kb = k >> 6, kk = k & 63;
  const int lane = ((kk >> 5) << 5) + rr;
  const int sub = (kk & 31) >> 3;
  return ((((size_t)rt * (Kp >> 6) + kb) * 4 + sub) * 64 + lane) * 8 + (kk & 7);
}

// Builds W_hi, W_lo (Mp x Kp bf16, zero padded) from positions in units of d.
__global__ void k_wm_build(const D4* __restrict__ pos, int n, __bf16* __restrict__ whi,
                           __bf16* __restrict__ wlo, int Mp, int Kp) {
  const int a = blockIdx.y;  // row
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= Mp || b >= Kp) return;
  const int i = a / 3, ca = a - 3 * (a / 3);
  const int j = b / 3, cb = b - 3 * (b / 3);
  double w = 0.0;
  if (i < n && j < n && i != j) {
    const D4 pi = pos[i], pj = pos[j];
    const double d[3] = {pj.x - pi.x, pj.y - pi.y, pj.z - pi.z};
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double inv = 1.0 / sqrt(r2);
    const double inv3 = inv * inv * inv;
    w = (3.0 * (d[ca] * inv) * (d[cb] * inv) - (ca == cb ? 1.0 : 0.0)) * inv3;
  }
  const __bf16 h = bf16_rn((float)w);
  const __bf16 l = bf16_rn((float)(w - (double)(float)h));
  whi[(size_t)a * Kp + b] = h;
  wlo[(size_t)a * Kp + b] = l;
}


__global__ __launch_bounds__(512) void k_wm_gemm(WMArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 Ws[2][2][WM_BN][WM_LD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  // block -> (W row tile, k split, replica tile); XCD-aware when the shape allows it:
  // an XCD (block index mod 8) owns whole W row tiles, both k splits and both replica
  // tiles, so each W slab is fetched from HBM once per step into that XCD's L2
  int rt, ks, ct;
  const int nb = g.n_rtiles * g.n_ctiles * WM_SK;
  if (g.n_ctiles == 2 && (g.n_rtiles & 7) == 0 && nb == (int)gridDim.x) {
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    rt = xcd * (g.n_rtiles >> 3) + (slot >> 2);
    ks = (slot >> 1) & 1;
    ct = slot & 1;
  } else {
    ct = blockIdx.x % g.n_ctiles;
    ks = (blockIdx.x / g.n_ctiles) % WM_SK;
    rt = blockIdx.x / (g.n_ctiles * WM_SK);
  }
  const int wrow0 = rt * WM_BN;           // first W row (output column) of the block
  const int rep0 = ct * WM_BM + w * 32;   // the wave's 32 replicas (output rows)
  const int kbeg = ks * (g.Kp / WM_SK);
  // M^T fragments of the wave's 32-replica tile (fragment-major layout, see mt_offset):
  // k-stage kb, substep s at ((tile * nkb + kb) * 4 + s) * 64 * 8 + lane * 8
  const int nkb = g.Kp >> 6;
  const size_t aoff = (size_t)(rep0 >> 5) * nkb * 4 * 64 * 8 + (size_t)lane * 8;
  const __bf16* ah = g.mhi + aoff;
  const __bf16* al = g.mlo + aoff;
  // W stage loads: 192 rows x 8 chunks of 8 bf16, hi and lo = 3072 chunks, 6 per thread
  // (rows tid/8 + 64 q for q = 0, 1, 2 of hi, then of lo), held in named registers (a
  // register array here would be moved to LDS)
  const int wr = tid >> 3, wk = (tid & 7) * 8;
  const __bf16* wsrc_h = g.whi + (size_t)(wrow0 + wr) * g.Kp + wk;
  const __bf16* wsrc_l = g.wlo + (size_t)(wrow0 + wr) * g.Kp + wk;
  const size_t wstep = (size_t)64 * g.Kp;  // 64 rows further for the next q
  uint4 w0, w1, w2, w3, w4, w5;
#define MH_LOAD_W(k0)                                                             \
  do {                                                                           \
    w0 = *reinterpret_cast<const uint4*>(wsrc_h + (k0));                         \
    w1 = *reinterpret_cast<const uint4*>(wsrc_h + wstep + (k0));                 \
    w2 = *reinterpret_cast<const uint4*>(wsrc_h + 2 * wstep + (k0));             \
    w3 = *reinterpret_cast<const uint4*>(wsrc_l + (k0));                         \
    w4 = *reinterpret_cast<const uint4*>(wsrc_l + wstep + (k0));                 \
    w5 = *reinterpret_cast<const uint4*>(wsrc_l + 2 * wstep + (k0));             \
  } while (0)
#define MH_STORE_W(buf)                                                          \
  do {                                                                           \
    *reinterpret_cast<uint4*>(&Ws[buf][0][wr][wk]) = w0;                         \
    *reinterpret_cast<uint4*>(&Ws[buf][0][wr + 64][wk]) = w1;                    \
    *reinterpret_cast<uint4*>(&Ws[buf][0][wr + 128][wk]) = w2;                   \
    *reinterpret_cast<uint4*>(&Ws[buf][1][wr][wk]) = w3;                         \
    *reinterpret_cast<uint4*>(&Ws[buf][1][wr + 64][wk]) = w4;                    \
    *reinterpret_cast<uint4*>(&Ws[buf][1][wr + 128][wk]) = w5;                   \
  } while (0)
  bf16x8 an[2][4];  // next stage M^T fragments [hi/lo][sub]
#define MH_LOAD_A(k0)                                                            \
  do {                                                                           \
    _Pragma("unroll") for (int s = 0; s < 4; ++s) {                              \
      an[0][s] = *reinterpret_cast<const bf16x8*>(ah + ((k0) >> 6) * 2048 + s * 512); \
      an[1][s] = *reinterpret_cast<const bf16x8*>(al + ((k0) >> 6) * 2048 + s * 512); \
    }                                                                            \
  } while (0)
  f32x16 acc[6];
#pragma unroll
  for (int u = 0; u < 6; ++u)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[u][e] = 0.f;

  const int nst = g.Kp / WM_SK / WM_BK;
  MH_LOAD_W(kbeg);
  MH_LOAD_A(kbeg);
  MH_STORE_W(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    bf16x8 ac[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int s = 0; s < 4; ++s) ac[h][s] = an[h][s];
    if (st + 1 < nst) {
      MH_LOAD_W(kbeg + (st + 1) * WM_BK);
      MH_LOAD_A(kbeg + (st + 1) * WM_BK);
    }
    // keep the next stage's loads in flight across the MFMAs: no memory operation may
    // move over this point, and the LDS stores of the next stage stay after them
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int kk = (lane >> 5) * 32 + s * 8;
      bf16x8 bh[6], bl[6];
#pragma unroll
      for (int u = 0; u < 6; ++u) {
        bh[u] = *reinterpret_cast<const bf16x8*>(&Ws[cur][0][u * 32 + (lane & 31)][kk]);
        bl[u] = *reinterpret_cast<const bf16x8*>(&Ws[cur][1][u * 32 + (lane & 31)][kk]);
      }
      // the three split products sweep the six accumulators in turn, so consecutive
      // MFMAs never depend on each other
#pragma unroll
      for (int u = 0; u < 6; ++u)
        acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ac[0][s], bh[u], acc[u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < 6; ++u)
        acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ac[1][s], bh[u], acc[u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < 6; ++u)
        acc[u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ac[0][s], bl[u], acc[u], 0, 0, 0);
    }
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    if (st + 1 < nst) {
      MH_STORE_W(cur ^ 1);
      __syncthreads();
    }
  }
#undef MH_LOAD_A
#undef MH_LOAD_W
#undef MH_STORE_W
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
template <bool kScan>
__global__ __launch_bounds__(256) void k_wm_update(const SysDesc* __restrict__ systems, WMArgs g,
                                                   const int64_t* __restrict__ kbase,
                                                   int64_t koff) {
  __shared__ double red[4];
  const int r = blockIdx.y;
  const SysDesc& s = systems[r];
  const int64_t k = (kbase ? *kbase : 0) + koff - s.k_origin;  // local step
  if (k < 0 || k >= s.total_steps) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int cur = (int)(k & 1);
  double mx = 0.0;
  if (i < s.n) {
    // partial products of the k splits, added in fixed order
    double fx = 0.0, fy = 0.0, fz = 0.0;
#pragma unroll
    for (int q = 0; q < WM_SK; ++q) {
      const float* f = g.bt + (size_t)q * g.Rp * g.Mp + (size_t)r * g.Mp + 3 * i;
      fx += (double)f[0];
      fy += (double)f[1];
      fz += (double)f[2];
    }
    mx = np_epilogue<kScan>(s, i, k, cur, fx, fy, fz);
    if (!s.field_only) {
      const D4 m = s.m64[(int64_t)(cur ^ 1) * s.stride + i];
      store_split(g, r, i, m.x, m.y, m.z);
    }
  }
  if (k >= s.kept0 && !s.field_only) {
    double v = mx;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0)
      s.recpart[(k - s.kept0) * s.ntiles + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
int wm_tile_rows() { return WM_BN; }
int wm_tile_reps() { return WM_BM; }
int wm_tile_k() { return WM_BK * WM_SK; }
int wm_ksplit() { return WM_SK; }

hipError_t launch_wm_build(const D4* pos, int n, __bf16* whi, __bf16* wlo, int Mp, int Kp,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_wm_build, dim3((Kp + 255) / 256, Mp), dim3(256), 0, st, pos, n, whi, wlo,
                     Mp, Kp);
  return hipGetLastError();
}

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

hipError_t launch_wm_pack(const SysDesc* d_sys, int R, int n, const WMArgs& g, int b,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_wm_pack, dim3((n + 255) / 256, R), dim3(256), 0, st, d_sys, g, b);
  return hipGetLastError();
}

}  // namespace mh
