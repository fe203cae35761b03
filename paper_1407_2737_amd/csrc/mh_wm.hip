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
// Tiling: block = 4 waves, tile = 256 replicas x 96 matrix rows, k-stage 64. The 96
// W rows of a stage (hi and lo) are staged through LDS (double buffered, rows padded
// to 72 bf16 so that 16-byte fragment reads do not conflict); each wave owns 64
// replicas and loads its M^T fragments straight from global memory, one stage ahead.
// Blocks are mapped so that the two replica tiles of a W row tile run on the same XCD
// (blockIdx mod 8), which fetches every W slab from HBM once per step.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mh_kernels.hpp"

namespace mh {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int WM_BM = 256;  // replicas per block
constexpr int WM_BN = 96;   // W rows per block
constexpr int WM_BK = 64;   // k per stage
constexpr int WM_LD = WM_BK + 8;

__device__ __forceinline__ __bf16 bf16_rn(float x) { return (__bf16)x; }

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


__global__ __launch_bounds__(256) void k_wm_gemm(WMArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 Ws[2][2][WM_BN][WM_LD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  // block -> (W row tile, replica tile); XCD-aware when the shape allows it
  int rt, ct;
  const int nb = g.n_rtiles * g.n_ctiles;
  if (g.n_ctiles == 2 && (g.n_rtiles & 7) == 0 && nb == (int)gridDim.x) {
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    rt = xcd * (g.n_rtiles >> 3) + (slot >> 1);
    ct = slot & 1;
  } else {
    rt = blockIdx.x / g.n_ctiles;
    ct = blockIdx.x - rt * g.n_ctiles;
  }
  const int wrow0 = rt * WM_BN;           // first W row (output column) of the block
  const int rep0 = ct * WM_BM + w * 64;   // first replica (output row) of this wave
  // M^T fragment sources of this lane: two 32-replica tiles, lane's replica row,
  // k = k0 + (lane/32)*32 + sub*8 + t
  const __bf16* ah[2];
  const __bf16* al[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const size_t off = (size_t)(rep0 + t * 32 + (lane & 31)) * g.Kp + (lane >> 5) * 32;
    ah[t] = g.mhi + off;
    al[t] = g.mlo + off;
  }
  // W stage loads: 96 rows x 8 chunks of 8 bf16, hi and lo = 1536 chunks, 6 per thread
  // (chunk c = tid + 256 q: rows 0..95 of hi for q < 3, of lo for q >= 3). The six
  // chunks are held in named registers; a register array here would be moved to LDS.
  const int wr = tid >> 3, wk = (tid & 7) * 8;
  const __bf16* wsrc_h = g.whi + (size_t)(wrow0 + wr) * g.Kp + wk;
  const __bf16* wsrc_l = g.wlo + (size_t)(wrow0 + wr) * g.Kp + wk;
  const size_t wstep = (size_t)32 * g.Kp;  // 32 rows further for the next q
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
    *reinterpret_cast<uint4*>(&Ws[buf][0][wr + 32][wk]) = w1;                    \
    *reinterpret_cast<uint4*>(&Ws[buf][0][wr + 64][wk]) = w2;                    \
    *reinterpret_cast<uint4*>(&Ws[buf][1][wr][wk]) = w3;                         \
    *reinterpret_cast<uint4*>(&Ws[buf][1][wr + 32][wk]) = w4;                    \
    *reinterpret_cast<uint4*>(&Ws[buf][1][wr + 64][wk]) = w5;                    \
  } while (0)
  bf16x8 an[2][2][4];  // next stage M^T fragments [tile][hi/lo][sub]
  auto load_a = [&](int k0) {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        an[t][0][s] = *reinterpret_cast<const bf16x8*>(ah[t] + k0 + s * 8);
        an[t][1][s] = *reinterpret_cast<const bf16x8*>(al[t] + k0 + s * 8);
      }
  };
  f32x16 acc[2][3];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[t][u][e] = 0.f;

  const int nst = g.Kp / WM_BK;
  MH_LOAD_W(0);
  load_a(0);
  MH_STORE_W(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int cur = st & 1;
    bf16x8 ac[2][2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int s = 0; s < 4; ++s) ac[t][h][s] = an[t][h][s];
    if (st + 1 < nst) {
      MH_LOAD_W((st + 1) * WM_BK);
      load_a((st + 1) * WM_BK);
    }
    // keep the next stage's loads in flight across the MFMAs: no memory operation may
    // move over this point, and the LDS stores of the next stage stay after them
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      bf16x8 bh[3], bl[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int r = u * 32 + (lane & 31);
        const int kk = (lane >> 5) * 32 + s * 8;
        bh[u] = *reinterpret_cast<const bf16x8*>(&Ws[cur][0][r][kk]);
        bl[u] = *reinterpret_cast<const bf16x8*>(&Ws[cur][1][r][kk]);
      }
      // the three split products sweep all six accumulators in turn, so consecutive
      // MFMAs never depend on each other
#pragma unroll
      for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int t = 0; t < 2; ++t)
          acc[t][u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ac[t][0][s], bh[u], acc[t][u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int t = 0; t < 2; ++t)
          acc[t][u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ac[t][1][s], bh[u], acc[t][u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < 3; ++u)
#pragma unroll
        for (int t = 0; t < 2; ++t)
          acc[t][u] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ac[t][0][s], bl[u], acc[t][u], 0, 0, 0);
    }
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    if (st + 1 < nst) {
      MH_STORE_W(cur ^ 1);
      __syncthreads();
    }
  }
#undef MH_LOAD_W
#undef MH_STORE_W
  // B^T[replica][W row]: lane holds column wrow0 + u*32 + lane%32 of rows
  // rep0 + t*32 + 8*(e/4) + 4*(lane/32) + e%4
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = rep0 + t * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        const int col = wrow0 + u * 32 + (lane & 31);
        g.bt[(size_t)row * g.Mp + col] = acc[t][u][e];
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
    g.mhi[(size_t)r * g.Kp + 3 * i + c] = h;
    g.mlo[(size_t)r * g.Kp + 3 * i + c] = l;
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
    const float* f = g.bt + (size_t)r * g.Mp + 3 * i;
    mx = np_epilogue(s, i, k, cur, (double)f[0], (double)f[1], (double)f[2]);
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
int wm_tile_k() { return WM_BK; }

hipError_t launch_wm_build(const D4* pos, int n, __bf16* whi, __bf16* wlo, int Mp, int Kp,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_wm_build, dim3((Kp + 255) / 256, Mp), dim3(256), 0, st, pos, n, whi, wlo,
                     Mp, Kp);
  return hipGetLastError();
}

hipError_t launch_wm_gemm(const WMArgs& g, hipStream_t st) {
  hipLaunchKernelGGL(k_wm_gemm, dim3(g.n_rtiles * g.n_ctiles), dim3(256), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_wm_update(const SysDesc* d_sys, int R, int n, const WMArgs& g,
                            const int64_t* kbase, int64_t koff, hipStream_t st) {
  hipLaunchKernelGGL(k_wm_update, dim3((n + 255) / 256, R), dim3(256), 0, st, d_sys, g, kbase,
                     koff);
  return hipGetLastError();
}

hipError_t launch_wm_pack(const SysDesc* d_sys, int R, int n, const WMArgs& g, int b,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_wm_pack, dim3((n + 255) / 256, R), dim3(256), 0, st, d_sys, g, b);
  return hipGetLastError();
}

}  // namespace mh
