// C-ABI runtime of mhkmc: validation, device memory, run orchestration and result
// retrieval. The arithmetic of the method runs in the kernels of mh_kernels.hip
// (and mh_wm.hip for the interaction-matrix form); this file only moves data and
// launches work.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <array>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <cstdio>
#include <cstring>
#include <new>
#include <unordered_map>
#include <vector>

#include "../../include/mhkmc.h"
#include "mh_kernels.hpp"

namespace mh {
hipError_t launch_resident(bool fp64, bool scan, const SysDesc* d_sys, int nsys, int64_t k0,
                           int64_t k1, int nmax, hipStream_t st);
size_t resident_lds_bytes(bool fp64, int nmax);
hipError_t set_resident_lds_limit();
int tile_width(int kind);
hipError_t launch_field(bool fp64, int kind, int G, const SysDesc* d_sys, const int4* d_tiles,
                        int ntiles, const int64_t* kbase, int64_t koff, hipStream_t st);
hipError_t launch_update(bool scan, const SysDesc* d_sys, const int2* d_blocks, int nblocks,
                         const int64_t* kbase, int64_t koff, hipStream_t st);
hipError_t launch_set_step(int64_t* kbase, int64_t v, bool add, hipStream_t st);
hipError_t launch_field_plan(const SysDesc& s, SysDesc* d_desc, int4* tiles, int tiles_per_part,
                             int nsplit, int2* ublocks, int nublocks, const double* m_in,
                             hipStream_t st);
hipError_t launch_field_out(const double* diag, double* B, int n, hipStream_t st);
hipError_t launch_empty_steps(int64_t steps, double* sink, hipStream_t st);
int wm_tile_rows();
int wm_tile_reps();
int wm_tile_k();
int wm_ksplit();
hipError_t launch_wm_gemm(const WMArgs& g, hipStream_t st);
hipError_t launch_wm_update(bool scan, const SysDesc* d_sys, int R, int n, const WMArgs& g,
                            const int64_t* kbase, int64_t koff, hipStream_t st);
hipError_t launch_wm_gemm_group(const WMGroupItem* d_items, int nitems, int nblocks,
                               hipStream_t st);
hipError_t launch_wm_update_group(bool scan, const SysDesc* d_all, const WMGroupItem* d_items,
                                  int nitems, int nblocks, const int64_t* kbase, int64_t koff,
                                  hipStream_t st);
hipError_t launch_wm_pack(const SysDesc* d_sys, int R, int n, const WMArgs& g, int b,
                          hipStream_t st);
hipError_t launch_finalize(const SysDesc* d_sys, int nsys, hipStream_t st);
hipError_t launch_init(const SysDesc* d_sys, int nsys, int nmax, hipStream_t st);
hipError_t launch_master(const SysDesc* d_sys, int nsys, int nmax, hipStream_t st);
hipError_t launch_local_conc(const D4* pos, int n, int N, double* phi, hipStream_t st);
hipError_t launch_sync32(const SysDesc* d_sys, int nsys, int nmax, int b, hipStream_t st);
hipError_t launch_finalize_asm(const double* d_sys_area, int R, double* d_out, hipStream_t st);
hipError_t launch_area_per_np(const double* d_area, int n, int R, int n_kept, double* d_out,
                              hipStream_t st);
hipError_t launch_philox_raw(uint64_t seed, uint64_t stream, const uint64_t* d_ctr, uint64_t* d_out,
                             int64_t nblk, hipStream_t st);
hipError_t launch_sw(const double* hx, const double* hy, const double* th0, double* out, int64_t n,
                     bool scan200, hipStream_t st);
}  // namespace mh

using namespace mh;

// Device scratch of the allocation-free field call (mh_field_noalloc): the plan, the
// moment copies, the partial field sums and the per-particle records of one Eq. 1
// evaluation. Every GPU the library runs on holds its own copy until the process ends.
// In host code this name is only a stand-in for the symbol: kernels receive the
// device address that hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr double kMu0 = 4e-7 * 3.14159265358979323846;
constexpr double kKB = 1.380649e-23;

// Device buffer that grows on demand.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  int ensure(size_t bytes) {
    if (bytes <= cap) return MH_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    if (hipMalloc(&p, bytes) != hipSuccess) return MH_ENOMEM;
    cap = bytes;
    return MH_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

struct PinBuf {
  void* p = nullptr;
  size_t cap = 0;
  int ensure(size_t bytes) {
    if (bytes <= cap) return MH_OK;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return MH_ENOMEM;
    cap = bytes;
    return MH_OK;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
  }
};

}  // namespace

// One autotuned launch shape of the tiled field kernel: for assemblies of the given
// precision class whose particle count and replica-group count fall in the buckets
// ending at n_max and groups_max, the tile width (0: 64 targets, 1: 16) and the
// blocks-per-CU target that sets the source split; us is the measured time per step.
struct ShapeEntry {
  int fp64;
  int64_t n_max, groups_max;
  int tile_kind, bpc;
  double us;
};

struct mh_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  // Input uploads (assembly creation). Non-blocking: a server's submit runs on the
  // caller's thread while the server thread may be capturing a graph on `stream`, and a
  // copy on the legacy stream would take an implicit dependency on that capture, which
  // the runtime rejects.
  hipStream_t upload = nullptr;
  // The resident systems of a run that also has tiled ones: their whole-run launch goes
  // here, forked from and joined back to the run's stream, so that it runs beside the
  // tiled steps instead of before them (created on first use).
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  int n_cu = 256;
  DevBuf d_sys;
  DevBuf d_probe;  // result of the empty-step timing kernel
  PinBuf h_stage;
  std::vector<unsigned char> staged;  // host image of the plan now in d_sys
  std::vector<hipGraphExec_t> timing_graphs;  // graphs of mh_time_kernels, kept to the end
  hipEvent_t tev[2] = {nullptr, nullptr};
  // optional per-launch timing of the step kernels (event pairs around each launch)
  int timing = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_kind;  // 0: tiled field, 1: resident run, 2: matrix step, 3: update
  // captured graph of G tiled steps, reused while the launch plan is unchanged
  DevBuf d_kbase;
  hipGraphExec_t gexec = nullptr;
  std::vector<uint64_t> gkey;
  int use_graphs = 1;
  std::vector<ShapeEntry> shapes;  // autotuned shapes (empty: the built-in rule)
  unsigned char* scratch = nullptr;  // this device's copy of `scratch` (device address)
  // recorded after the last launch of a run that reads the plan in d_sys / d_kbase (or
  // the captured graph): the next run, on any stream, waits for it before re-staging
  hipEvent_t plan_done = nullptr;
  bool plan_pending = false;
};

struct mh_asm {
  mh_ctx* ctx = nullptr;
  int64_t n = 0;
  int64_t n_axes_sets = 1;
  int64_t n_pos_sets = 1;  // replica r uses position set r mod n_pos_sets
  mh_params p{};
  // geometry
  DevBuf pos64, pos32, axes;
  // run state
  int64_t R = 0;
  uint64_t seed = 0;
  bool ran = false;
  int ntiles = 1;
  int resident = 0;
  int tile_kind = 0;  // 0: 64 targets per block, 1: 16
  int nsplit = 1;     // source parts per field tile
  int rec_slots = 1;  // loop record partial sums per update block (rec_slots_for)
  DevBuf m64, m32, area, recpart, rec, sys_area, stats, diag, tmp, field, dhdip;
  // interaction-matrix form (W generated in the product kernel): M^T hi/lo (Rp x Kp),
  // B^T partial sums (k splits x Rp x Mp)
  DevBuf mhi, mlo, bt;
  int Mp = 0, Kp = 0, Rp = 0;
  int state_parity = 0;  // the current moments live in buffer state_parity
  int64_t k_origin = 0;    // global step of local step 0 (continuous batching)
  int force_kind = -1, force_bpc = 0;  // autotuner candidates (-1: table or rule)
  std::vector<double> hmax;  // per-replica field amplitudes (replica r uses r mod size)
  uint64_t stream_base = 0;  // Philox stream of replica 0
  hipEvent_t done = nullptr;
  // host copy of the per-run system descriptors (for diagnostics re-runs)
};

namespace {

// Device address of `scratch` on `device`, resolved once per device with that device
// current (each GPU holds the array at its own address).
std::mutex g_scratch_mu;
std::unordered_map<int, unsigned char*> g_scratch_addr;
int scratch_address(int device, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it == g_scratch_addr.end()) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MH_EDEVICE;
    it = g_scratch_addr.emplace(device, static_cast<unsigned char*>(p)).first;
  }
  *out = it->second;
  return MH_OK;
}

inline int set_dev(mh_ctx* c) {
  return hipSetDevice(c->device) == hipSuccess ? MH_OK : MH_EDEVICE;
}

// The context's plan staging (pinned stage, d_sys, d_kbase, graph) is shared by all its
// runs, whatever stream they use: wait until the previous run no longer reads it.
int wait_plan_free(mh_ctx* c) {
  if (c->plan_pending && hipEventSynchronize(c->plan_done) != hipSuccess) return MH_EDEVICE;
  c->plan_pending = false;
  return MH_OK;
}
int mark_plan_busy(mh_ctx* c, hipStream_t st) {
  if (!c->plan_done && hipEventCreateWithFlags(&c->plan_done, hipEventDisableTiming) != hipSuccess)
    return MH_EDEVICE;
  if (hipEventRecord(c->plan_done, st) != hipSuccess) return MH_EDEVICE;
  c->plan_pending = true;
  return MH_OK;
}
// An assembly's buffers may be reallocated by its next run: wait for its last one.
int wait_asm_idle(mh_asm* a) {
  if (a->ran && a->done && hipEventSynchronize(a->done) != hipSuccess) return MH_EDEVICE;
  return MH_OK;
}

int total_steps(const mh_params& p) { return p.n_periods * p.steps_per_period; }
int kept0(const mh_params& p) { return p.n_discard * p.steps_per_period; }
int n_kept(const mh_params& p) { return p.n_periods - p.n_discard; }

int validate_params(const mh_params* p) {
  if (!p) return MH_EINVAL;
  const double v[] = {p->Ms,      p->Keff,         p->d,           p->T,
                      p->tau0,    p->rho,          p->f,           p->mu0Hmax,
                      p->dt_override, p->field_dir[0], p->field_dir[1], p->field_dir[2]};
  for (double x : v)
    if (!std::isfinite(x)) return MH_EINVAL;
  if (p->Ms <= 0 || p->Keff < 0 || p->d <= 0 || p->T < 0 || p->tau0 <= 0 || p->rho <= 0 ||
      p->f <= 0 || p->mu0Hmax < 0 || p->dt_override < 0)
    return MH_EINVAL;
  if (p->steps_per_period < 2 || (p->steps_per_period & 1)) return MH_EINVAL;
  if (p->n_periods < 1 || p->n_discard < 0 || p->n_discard >= p->n_periods) return MH_EINVAL;
  if ((int64_t)p->n_periods * p->steps_per_period > (int64_t)1 << 30) return MH_EINVAL;
  if (p->prob_form != MH_P_TWO_STATE && p->prob_form != MH_P_SINGLE_RATE) return MH_EINVAL;
  if (p->precision != MH_FP64 && p->precision != MH_FP32_FIELD && p->precision != MH_BF16X3_WM)
    return MH_EINVAL;
  if (p->interactions != 0 && p->interactions != 1) return MH_EINVAL;
  if (p->extrema_mode != MH_EXTREMA_EXACT && p->extrema_mode != MH_EXTREMA_SCAN200)
    return MH_EINVAL;
  if (p->reserved) return MH_EINVAL;
  return MH_OK;
}

// Pairs closer than d (1 - 1e-9): cell list with cell size d.
int check_overlap(int64_t n, const double* pos, double d) {
  const double lim = d * (1.0 - 1e-9);
  const double lim2 = lim * lim;
  double lo[3] = {INFINITY, INFINITY, INFINITY};
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) lo[c] = std::min(lo[c], pos[3 * i + c]);
  std::unordered_map<int64_t, std::vector<int64_t>> cells;
  cells.reserve((size_t)n * 2);
  auto key = [](int64_t a, int64_t b, int64_t c) {
    return (a & 0x1FFFFF) | ((b & 0x1FFFFF) << 21) | ((c & 0x1FFFFF) << 42);
  };
  for (int64_t i = 0; i < n; ++i) {
    const int64_t cx = (int64_t)std::floor((pos[3 * i] - lo[0]) / d);
    const int64_t cy = (int64_t)std::floor((pos[3 * i + 1] - lo[1]) / d);
    const int64_t cz = (int64_t)std::floor((pos[3 * i + 2] - lo[2]) / d);
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          auto it = cells.find(key(cx + dx, cy + dy, cz + dz));
          if (it == cells.end()) continue;
          for (int64_t j : it->second) {
            const double ex = pos[3 * j] - pos[3 * i], ey = pos[3 * j + 1] - pos[3 * i + 1],
                         ez = pos[3 * j + 2] - pos[3 * i + 2];
            if (ex * ex + ey * ey + ez * ez < lim2) return MH_EOVERLAP;
          }
        }
    cells[key(cx, cy, cz)].push_back(i);
  }
  return MH_OK;
}

// Launch form of an assembly, decided from its own size and replica count only, so
// that its results do not depend on what else runs in the same batch.
bool wants_resident(const mh_asm* a, int64_t R) {
  if (a->p.precision == MH_BF16X3_WM) return false;
  const bool fp64 = a->p.precision == MH_FP64;
  if (a->n <= 256) return true;
  // a single workgroup per replica pays off once its replicas fill the device
  return R >= 4 * a->ctx->n_cu && a->n <= (fp64 ? 512 : 1024);
}

// Buckets of the shape table: particle counts and replica groups (field blocks share
// the pair geometry across up to four FP32 replicas; FP64 groups are single replicas).
int64_t n_bucket(int64_t n) {
  int64_t b = 256;
  while (b < n && b < ((int64_t)1 << 40)) b *= 2;
  return b;
}
int64_t g_bucket(int64_t g) {
  int64_t b = 1;
  while (b < g && b < ((int64_t)1 << 40)) b *= 4;
  return b;
}
int64_t groups_of(const mh_asm* a, int64_t R) {
  if (a->p.precision == MH_FP64) return R;
  // FP32 groups of up to four replicas that share a position set
  int64_t g = 0;
  const int64_t P = std::min<int64_t>(a->n_pos_sets, R);
  for (int64_t q = 0; q < P; ++q) g += ((R - q + P - 1) / P + 3) / 4;
  return g;
}

// Launch shape of the tiled field kernel: an autotuner candidate, else the context's
// autotuned entry for the assembly's buckets, else the built-in rule: 64 targets per
// block once the assembly's own blocks fill the device (else 16, four times more
// blocks), and a source split for about three blocks per CU. The rule's constants
// were measured on one 5000-particle assembly with three replicas and on a batch of
// 256 assemblies of 200-8000 particles (three per CU beat two, four and six on both).
// Every input is the assembly's own (N, replicas, precision) and the context's
// table, so an assembly's result does not depend on the batch it runs in.
struct Shape {
  int kind, bpc;
};
Shape shape_for(const mh_asm* a, int64_t R) {
  if (a->force_kind >= 0) return Shape{a->force_kind, a->force_bpc};
  const int64_t groups = groups_of(a, R);
  const int fp64 = a->p.precision == MH_FP64 ? 1 : 0;
  const int64_t nb = n_bucket(a->n), gb = g_bucket(groups);
  for (const ShapeEntry& e : a->ctx->shapes)
    if (e.fp64 == fp64 && e.n_max == nb && e.groups_max == gb) return Shape{e.tile_kind, e.bpc};
  return Shape{groups * ((a->n + 63) / 64) >= a->ctx->n_cu ? 0 : 1, 3};
}

int tile_kind_for(const mh_asm* a, int64_t R) { return shape_for(a, R).kind; }

// Source parts per field tile: enough blocks for the shape's blocks per CU, with parts
// of at least 1250 sources so that every block keeps enough work to cover its staging
// and reduction.
int nsplit_for(const mh_asm* a, int64_t R, int kind) {
  const int64_t groups = groups_of(a, R);
  const int64_t TI = kind == 0 ? 64 : 16;
  const int64_t blocks = groups * ((a->n + TI - 1) / TI);
  int64_t sp = ((int64_t)shape_for(a, R).bpc * a->ctx->n_cu + blocks - 1) / blocks;
  sp = std::min<int64_t>(sp, std::max<int64_t>(1, a->n / 1250));
  return (int)std::max<int64_t>(1, std::min<int64_t>(sp, 16));
}

// (Re)allocate a replica set and its per-run buffers.
int prepare_run(mh_asm* a, int64_t R, uint64_t seed, bool resident, int tile_kind) {
  const int64_t n = a->n;
  a->resident = resident ? 1 : 0;
  a->tile_kind = tile_kind;
  a->nsplit = resident ? 1 : nsplit_for(a, R, tile_kind);
  a->ntiles = resident ? 1 : (int)((n + 255) / 256);
  const int64_t rows = (int64_t)n_kept(a->p) * a->p.steps_per_period;
  int e;
  if ((e = a->m64.ensure(sizeof(D4) * 2 * R * n))) return e;
  if (a->p.precision == MH_FP32_FIELD && (e = a->m32.ensure(sizeof(F4) * 2 * R * n))) return e;
  if ((e = a->area.ensure(sizeof(double) * 2 * R * n))) return e;
  if ((e = a->dhdip.ensure(sizeof(double) * R * n))) return e;
  a->rec_slots = rec_slots_for(R, a->ntiles);
  if ((e = a->recpart.ensure(sizeof(double) * R * rows * a->ntiles * a->rec_slots + 8))) return e;
  if ((e = a->rec.ensure(sizeof(double) * R * rows + 8))) return e;
  if ((e = a->sys_area.ensure(sizeof(double) * R))) return e;
  if ((e = a->stats.ensure(sizeof(double) * 4))) return e;
  const bool wm = a->p.precision == MH_BF16X3_WM;
  // partial field sums: FP32 for the FP32 field form, FP64 otherwise
  const size_t part_bytes = a->p.precision == MH_FP32_FIELD ? sizeof(F4) : sizeof(D4);
  if (!resident && !wm && (e = a->field.ensure(part_bytes * R * n * a->nsplit))) return e;
  if (wm) {
    {
      const int64_t rows = 3 * n;
      const int64_t rq = 8 * wm_tile_rows();  // whole row tiles, a multiple of 8 for the XCD map
      a->Mp = (int)((rows + rq - 1) / rq * rq);
      a->Kp = (int)((rows + wm_tile_k() - 1) / wm_tile_k() * wm_tile_k());
    }
    const int rt = wm_tile_reps();
    const int Rp = (int)((R + rt - 1) / rt * rt);
    const size_t mb = sizeof(__bf16) * (size_t)Rp * a->Kp;
    if (Rp != a->Rp || !a->mhi.p) {
      a->mhi.release();
      a->mlo.release();
      if ((e = a->mhi.ensure(mb)) || (e = a->mlo.ensure(mb))) return e;
      if (hipMemset(a->mhi.p, 0, mb) != hipSuccess || hipMemset(a->mlo.p, 0, mb) != hipSuccess)
        return MH_EDEVICE;
      a->Rp = Rp;
    }
    if ((e = a->bt.ensure(sizeof(float) * (size_t)wm_ksplit() * Rp * a->Mp))) return e;
  }
  a->R = R;
  a->seed = seed;
  return MH_OK;
}

// Material, field and protocol part of replica r's descriptor (no run buffers).
SysDesc desc_physics(const mh_asm* a, int64_t r) {
  const mh_params& p = a->p;
  SysDesc s{};
  const int64_t n = a->n;
  const int64_t pset = r % a->n_pos_sets;
  s.pos64 = a->pos64.as<D4>() + pset * n;
  s.pos32 = a->pos32.as<F4>() + pset * n;
  s.axes = a->axes.as<D4>() + (r % a->n_axes_sets) * n;
  const double V = 3.14159265358979323846 * p.d * p.d * p.d / 6.0;
  s.np.BK = p.Keff > 0 ? 2.0 * p.Keff / p.Ms : 0.0;
  s.np.BK_inv = p.Keff > 0 ? p.Ms / (2.0 * p.Keff) : 0.0;
  s.np.beta = p.T > 0 ? p.Keff * V / (kKB * p.T) : 0.0;
  const double dt = p.dt_override > 0 ? p.dt_override : 1.0 / (p.f * p.steps_per_period);
  s.np.nu0dt = dt / p.tau0;
  s.np.prob_form = p.prob_form;
  s.np.scan200 = p.extrema_mode == MH_EXTREMA_SCAN200 ? 1 : 0;
  s.np.thermal = p.T > 0 ? 1 : 0;
  s.np.aniso = p.Keff > 0 ? 1 : 0;
  s.Bmax = a->hmax.empty() ? p.mu0Hmax : a->hmax[(size_t)(r % (int64_t)a->hmax.size())];
  s.Bscale = p.interactions ? kMu0 * p.Ms / 24.0 : 0.0;
  {
    const double* e = p.field_dir;
    const double en = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    s.eh[0] = en == 0.0 ? 1.0 : e[0] / en;
    s.eh[1] = en == 0.0 ? 0.0 : e[1] / en;
    s.eh[2] = en == 0.0 ? 0.0 : e[2] / en;
  }
  s.Ms = p.Ms;
  s.n = (int32_t)n;
  s.S = p.steps_per_period;
  s.total_steps = total_steps(p);
  s.kept0 = kept0(p);
  s.static_field = p.dt_override > 0 ? 1 : 0;
  s.field_only = 0;
  return s;
}

SysDesc make_desc(const mh_asm* a, int64_t r) {
  const mh_params& p = a->p;
  SysDesc s = desc_physics(a, r);
  const int64_t n = a->n;
  s.m64 = a->m64.as<D4>() + r * n;
  // FP32 moment copies exist only for the FP32 field form, which is their one reader
  s.m32 = a->p.precision == MH_FP32_FIELD ? a->m32.as<F4>() + r * n : nullptr;
  s.area = a->area.as<double>() + r * 2 * n;
  const int64_t rows = (int64_t)n_kept(p) * p.steps_per_period;
  s.recpart = a->recpart.as<double>() + r * rows * a->ntiles * a->rec_slots;
  s.rec_slots = a->rec_slots;
  s.rec = a->rec.as<double>() + r * rows;
  const bool f32 = a->p.precision == MH_FP32_FIELD;
  s.field = a->resident || f32 ? nullptr : a->field.as<D4>() + r * n * a->nsplit;
  s.field32 = a->resident || !f32 ? nullptr : a->field.as<F4>() + r * n * a->nsplit;
  // without interactions no dipolar sum is formed: no field tiles, and the update
  // reads no partial sums (its dipolar part is exactly zero)
  s.nsplit = a->p.interactions ? a->nsplit : 0;
  s.sys_area = a->sys_area.as<double>() + r;
  s.dhdip = a->dhdip.as<double>() + r * n;
  s.diag = nullptr;
  s.stride = a->R * n;
  s.seed = a->seed;
  s.stream = a->stream_base + (uint64_t)r;
  s.k_origin = a->k_origin;
  s.ntiles = a->ntiles;
  return s;
}

WMArgs wm_args(const mh_asm* a) {
  WMArgs g{};
  g.pos = a->pos64.as<D4>();
  g.n = (int)a->n;
  g.mhi = a->mhi.as<__bf16>();
  g.mlo = a->mlo.as<__bf16>();
  g.bt = a->bt.as<float>();
  g.Mp = a->Mp;
  g.Kp = a->Kp;
  g.Rp = a->Rp;
  g.n_rtiles = a->Mp / wm_tile_rows();
  g.n_ctiles = a->Rp / wm_tile_reps();
  return g;
}

struct WMItem {
  mh_asm* a;
  int first;  // index of replica 0 in the all-systems list
  WMArgs g;
};

// field launch groups: precision x tile kind x replicas per block (1..4)
constexpr int kGroups = 2 * 2 * 4;
inline int gidx(int fp64, int kind, int G) { return (fp64 * 2 + kind) * 4 + (G - 1); }

struct Plan {
  std::vector<SysDesc> res64, res32, til[kGroups];
  std::vector<int4> tiles[kGroups];
  std::vector<WMItem> wm;
  // two or more matrix-form systems: one product launch and one update launch per
  // extremum mode cover them all (wmu[1]: the 200-point scan)
  std::vector<WMGroupItem> wmg, wmu[2];
  int wmg_blocks = 0, wmu_blocks[2] = {0, 0};
  bool wm_grouped = false;
  std::vector<SysDesc> upd;   // all tiled systems
  std::vector<int2> ublocks;  // (system in upd, block of 256 particles)
  int nmax_res64 = 0, nmax_res32 = 0;
  int64_t kmax = 0;
  int nmax_all = 0;
  // a system in the list takes step iv as the 200-point scan: launch the kernel
  // instantiation that carries it
  bool scan_res64 = false, scan_res32 = false, scan_upd = false;
};

// The R replicas of one tiled assembly: field blocks take up to 4 replicas at a time in
// FP32 (they share positions, so the pair geometry is computed once for all of them).
// Field tiles of one assembly's replicas: FP32 replicas that share a position set
// (replica r has set r mod P) are grouped four at a time, in replica order within a
// set, so that a block applies one pair geometry to each group member's moments.
void add_tiled(Plan& pl, int fp64, int kind, const std::vector<SysDesc>& reps, int64_t P) {
  const int R = (int)reps.size();
  const int TI = tile_width(kind);
  const int Gmax = fp64 ? 1 : 4;
  P = std::max<int64_t>(1, std::min<int64_t>(P, R));
  for (int64_t q = 0; q < P; ++q) {
    std::vector<int> mem;
    for (int r = (int)q; r < R; r += (int)P) mem.push_back(r);
    for (size_t g0 = 0; g0 < mem.size(); g0 += Gmax) {
      const int gn = (int)std::min<size_t>(Gmax, mem.size() - g0);
      const int gi = gidx(fp64, kind, gn);
      const int sidx = (int)pl.til[gi].size();
      for (int r = 0; r < gn; ++r) pl.til[gi].push_back(reps[mem[g0 + r]]);
      // part-major: the last part of each tile, the shortest, is dispatched last
      const int n = reps[0].n;
      for (int part = 0; part < reps[0].nsplit; ++part)
        for (int it = 0; it < (n + TI - 1) / TI; ++it)
          pl.tiles[gi].push_back(int4{sidx, it, gn, part});
    }
  }
  for (const SysDesc& s : reps) {
    const int uidx = (int)pl.upd.size();
    pl.upd.push_back(s);
    for (int b = 0; b < s.ntiles; ++b) pl.ublocks.push_back(int2{uidx, b});
  }
}

// Block ranges of the grouped matrix-form launches. Products go longest first (the
// longest k range, then the most blocks), each range starting at a multiple of 8 so that
// every block keeps its XCD; updates go largest first. A block's work is the same as
// in the system's own launch, so the results do not depend on the grouping. Returns
// false (no grouping: one launch per system) where a grouped grid would exceed the
// one-dimensional grid's range.
bool group_wm(Plan& pl) {
  int64_t tot_g = 0, tot_u = 0;
  for (const WMItem& it : pl.wm) {
    tot_g += ((int64_t)it.g.n_rtiles * it.g.n_ctiles * wm_ksplit() + 7) / 8 * 8;
    tot_u += (it.a->n + 255) / 256 * it.a->R;
  }
  if (tot_g > ((int64_t)1 << 30) || tot_u > ((int64_t)1 << 30)) return false;
  std::vector<int> ord(pl.wm.size());
  for (size_t q = 0; q < ord.size(); ++q) ord[q] = (int)q;
  auto gemm_blocks = [](const WMArgs& g) { return g.n_rtiles * g.n_ctiles * wm_ksplit(); };
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
    const WMArgs &a = pl.wm[x].g, &b = pl.wm[y].g;
    return a.Kp != b.Kp ? a.Kp > b.Kp : gemm_blocks(a) > gemm_blocks(b);
  });
  for (int q : ord) {
    const WMItem& it = pl.wm[q];
    WMGroupItem x{};
    x.g = it.g;
    x.boff = pl.wmg_blocks;
    x.nb = gemm_blocks(it.g);
    pl.wmg.push_back(x);
    pl.wmg_blocks += (x.nb + 7) / 8 * 8;
  }
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
    return pl.wm[x].a->n * pl.wm[x].a->R > pl.wm[y].a->n * pl.wm[y].a->R;
  });
  for (int q : ord) {
    const WMItem& it = pl.wm[q];
    const int sc = it.a->p.extrema_mode == MH_EXTREMA_SCAN200 ? 1 : 0;
    WMGroupItem x{};
    x.g = it.g;
    x.first = it.first;
    x.nbx = (int)((it.a->n + 255) / 256);
    x.nb = x.nbx * (int)it.a->R;
    x.boff = pl.wmu_blocks[sc];
    pl.wmu[sc].push_back(x);
    pl.wmu_blocks[sc] += x.nb;
  }
  return true;
}

// Host image of a run's plan: arrays placed at 256-byte aligned offsets of one blob,
// uploaded to the context's d_sys in a single copy. An empty array has no place.
constexpr size_t kNoPlace = ~(size_t)0;
struct PlanBlob {
  std::vector<unsigned char> h;
  template <typename T>
  size_t put(const std::vector<T>& v) {
    if (v.empty()) return kNoPlace;
    const size_t off = (h.size() + 255) & ~(size_t)255;
    h.resize(off + sizeof(T) * v.size(), 0);
    std::memcpy(h.data() + off, v.data(), sizeof(T) * v.size());
    return off;
  }
};
template <typename T>
T* blob_ptr(mh_ctx* c, size_t off) {
  return off == kNoPlace ? nullptr : reinterpret_cast<T*>(c->d_sys.as<char>() + off);
}

// Event pair around a launch when timing is on; returns the index of the pair or -1.
int timing_begin(mh_ctx* c, hipStream_t st, int kind) {
  if (!c->timing) return -1;
  if (c->ev_used + 2 > c->ev_pool.size()) {
    for (int q = 0; q < 512; ++q) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      c->ev_pool.push_back(e);
    }
  }
  const int idx = (int)c->ev_used;
  c->ev_used += 2;
  c->ev_kind.push_back(kind);
  (void)hipEventRecord(c->ev_pool[idx], st);
  return idx;
}
void timing_end(mh_ctx* c, hipStream_t st, int idx) {
  if (idx >= 0) (void)hipEventRecord(c->ev_pool[idx + 1], st);
}

struct RunOpts {
  bool init = true;          // fresh run: initial moments, zero accumulators
  bool sync32 = true;        // refresh FP32 moment copies (moments written from the host)
  int64_t k0 = 0, k1 = -1;   // step range (-1: to the end)
  bool finalize = true;
  bool field_only = false;
  double* diag = nullptr;    // device diag buffer base (per asm: R*n*8)
  // launch timing instead of a run: kernels of one kind (0 field sums, 2 matrix product,
  // 3 update, 4 matrix-form update) for local steps time_k0 .. + time_launches-1, replayed
  // back to back from a captured graph; mean microseconds per step into *time_us
  int time_kind = -1;
  int time_launches = 0, time_reps = 0;
  int64_t time_k0 = 0;  // first local step of the timed launches
  double* time_us = nullptr;
};

// Mean duration of `unit` (the launches of one step of one kernel kind): L units for
// local steps kstart .. kstart+L-1 are captured once into a graph, replayed once to warm up, then
// `reps` times between two events on the stream. The graph is kept until the context is
// destroyed, so timing creates no destroy/instantiate churn between runs.
template <typename F>
int time_graph(mh_ctx* c, hipStream_t st, int64_t kstart, int L, int reps, F&& unit, double* us) {
  int e;
  if ((e = c->d_kbase.ensure(sizeof(int64_t)))) return e;
  int64_t* kb = c->d_kbase.as<int64_t>();
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return MH_EDEVICE;
  int rc = MH_OK;
  for (int j = 0; j < L && rc == MH_OK; ++j) rc = unit(kb, j);
  if (hipStreamEndCapture(st, &g) != hipSuccess || rc != MH_OK) {
    if (g) (void)hipGraphDestroy(g);
    return MH_EDEVICE;
  }
  const hipError_t ie = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) return MH_EDEVICE;
  c->timing_graphs.push_back(x);
  if (!c->tev[0] && (hipEventCreate(&c->tev[0]) != hipSuccess || hipEventCreate(&c->tev[1]) != hipSuccess))
    return MH_EDEVICE;
  if (launch_set_step(kb, kstart, false, st) != hipSuccess || hipGraphLaunch(x, st) != hipSuccess ||
      hipEventRecord(c->tev[0], st) != hipSuccess)
    return MH_EDEVICE;
  for (int q = 0; q < reps; ++q)
    if (hipGraphLaunch(x, st) != hipSuccess) return MH_EDEVICE;
  float ms = 0.f;
  if (hipEventRecord(c->tev[1], st) != hipSuccess || hipEventSynchronize(c->tev[1]) != hipSuccess ||
      hipEventElapsedTime(&ms, c->tev[0], c->tev[1]) != hipSuccess)
    return MH_EDEVICE;
  *us = (double)ms * 1e3 / ((double)L * reps);
  return MH_OK;
}

int run_systems(std::vector<mh_asm*>& asms, const std::vector<int64_t>& Rs,
                const std::vector<uint64_t>& seeds, hipStream_t st, const RunOpts& o) {
  if (asms.empty()) return MH_OK;
  mh_ctx* c = asms[0]->ctx;
  for (auto* a : asms)
    if (a->ctx != c) return MH_EINVAL;
  if (set_dev(c)) return MH_EDEVICE;
  if (!st) st = c->stream;

  Plan pl;
  std::vector<std::pair<mh_asm*, std::pair<int, int>>> fin;  // asm -> range in all-sys list
  std::vector<SysDesc> all;
  for (size_t q = 0; q < asms.size(); ++q) {
    mh_asm* a = asms[q];
    if (o.init) {
      int e = wait_asm_idle(a);
      if (!e) e = prepare_run(a, Rs[q], seeds[q], wants_resident(a, Rs[q]), tile_kind_for(a, Rs[q]));
      if (e) return e;
    }
    const bool fp64 = a->p.precision == MH_FP64;
    const int first = (int)all.size();
    std::vector<SysDesc> reps;
    for (int64_t r = 0; r < a->R; ++r) {
      SysDesc s = make_desc(a, r);
      s.field_only = o.field_only ? 1 : 0;
      if (o.diag) s.diag = o.diag + r * a->n * 8;
      all.push_back(s);
      if (a->p.precision == MH_BF16X3_WM) {
        // handled by the matrix path below
      } else if (a->resident) {
        (fp64 ? pl.res64 : pl.res32).push_back(s);
        (fp64 ? pl.scan_res64 : pl.scan_res32) |= s.np.scan200 != 0;
        int& nm = fp64 ? pl.nmax_res64 : pl.nmax_res32;
        nm = std::max(nm, (int)a->n);
      } else {
        reps.push_back(s);
        pl.scan_upd |= s.np.scan200 != 0;
      }
      pl.kmax = std::max<int64_t>(pl.kmax, s.k_origin + s.total_steps);
      pl.nmax_all = std::max(pl.nmax_all, (int)a->n);
    }
    if (!reps.empty()) add_tiled(pl, fp64 ? 1 : 0, a->tile_kind, reps, a->n_pos_sets);
    fin.push_back({a, {first, (int)all.size()}});
    if (a->p.precision == MH_BF16X3_WM) pl.wm.push_back(WMItem{a, first, wm_args(a)});
  }
  if (pl.wm.size() >= 2) pl.wm_grouped = group_wm(pl);
  // descriptors and tile lists, laid out as one blob; a plan identical to the one the
  // context staged last (a server chunk of the same requests) is not uploaded again
  PlanBlob blob;
  const size_t o_all = blob.put(all), o_res64 = blob.put(pl.res64), o_res32 = blob.put(pl.res32);
  size_t o_til[kGroups], o_tiles[kGroups];
  for (int gi = 0; gi < kGroups; ++gi) {
    o_til[gi] = blob.put(pl.til[gi]);
    o_tiles[gi] = blob.put(pl.tiles[gi]);
  }
  const size_t o_upd = blob.put(pl.upd), o_ublocks = blob.put(pl.ublocks);
  const size_t o_wmg = blob.put(pl.wmg), o_wmu0 = blob.put(pl.wmu[0]), o_wmu1 = blob.put(pl.wmu[1]);
  const size_t off = blob.h.size();
  int e;
  if (!(c->d_sys.p && off <= c->d_sys.cap && blob.h == c->staged)) {
    if ((e = wait_plan_free(c))) return e;  // stage reuse, whichever stream ran last
    if (hipStreamSynchronize(st) != hipSuccess) return MH_EDEVICE;
    if ((e = c->h_stage.ensure(off + 256)) || (e = c->d_sys.ensure(off + 256))) return e;
    if (off) {
      std::memcpy(c->h_stage.p, blob.h.data(), off);
      if (hipMemcpyAsync(c->d_sys.p, c->h_stage.p, off, hipMemcpyHostToDevice, st) != hipSuccess)
        return MH_EDEVICE;
    }
    c->staged.swap(blob.h);
  }
  SysDesc* d_all = blob_ptr<SysDesc>(c, o_all);
  SysDesc* d_res64 = blob_ptr<SysDesc>(c, o_res64);
  SysDesc* d_res32 = blob_ptr<SysDesc>(c, o_res32);
  SysDesc* d_til[kGroups];
  int4* d_tiles[kGroups];
  for (int gi = 0; gi < kGroups; ++gi) {
    d_til[gi] = blob_ptr<SysDesc>(c, o_til[gi]);
    d_tiles[gi] = blob_ptr<int4>(c, o_tiles[gi]);
  }
  SysDesc* d_upd = blob_ptr<SysDesc>(c, o_upd);
  int2* d_ublocks = blob_ptr<int2>(c, o_ublocks);
  WMGroupItem* d_wmg = blob_ptr<WMGroupItem>(c, o_wmg);
  WMGroupItem* d_wmu[2] = {blob_ptr<WMGroupItem>(c, o_wmu0), blob_ptr<WMGroupItem>(c, o_wmu1)};
  // the matrix-form launches of one step: kind 2 the products, kind 4 the updates
  auto wm_launches = [&](int kind, const int64_t* kb, int64_t koff) -> hipError_t {
    hipError_t r = hipSuccess;
    if (pl.wm_grouped) {
      if (kind == 2) return launch_wm_gemm_group(d_wmg, (int)pl.wmg.size(), pl.wmg_blocks, st);
      for (int sc = 0; sc < 2 && r == hipSuccess; ++sc)
        if (!pl.wmu[sc].empty())
          r = launch_wm_update_group(sc == 1, d_all, d_wmu[sc], (int)pl.wmu[sc].size(),
                                     pl.wmu_blocks[sc], kb, koff, st);
      return r;
    }
    for (auto& it : pl.wm) {
      if (r != hipSuccess) break;
      r = kind == 2 ? launch_wm_gemm(it.g, st)
                    : launch_wm_update(it.a->p.extrema_mode == MH_EXTREMA_SCAN200, d_all + it.first,
                                       (int)it.a->R, (int)it.a->n, it.g, kb, koff, st);
    }
    return r;
  };
  if (o.init) {
    if (launch_init(d_all, (int)all.size(), pl.nmax_all, st) != hipSuccess) return MH_EDEVICE;
  } else if (o.sync32) {
    // moments may have been replaced from the host: refresh the FP32 copies
    if (launch_sync32(d_all, (int)all.size(), pl.nmax_all, (int)(o.k0 & 1), st) != hipSuccess)
      return MH_EDEVICE;
  }
  if (o.init || o.sync32)
    for (auto& it : pl.wm)
      if (launch_wm_pack(d_all + it.first, (int)it.a->R, (int)it.a->n, it.g,
                         (int)((o.k0 - it.a->k_origin) & 1), st) != hipSuccess)
        return MH_EDEVICE;
  if (o.time_kind >= 0) {
    auto unit = [&](const int64_t* kb, int64_t koff) -> int {
      hipError_t r = hipSuccess;
      if (o.time_kind == 0) {
        for (int f = 0; f < 2; ++f)
          for (int kd = 0; kd < 2; ++kd)
            for (int G = 1; G <= 4 && r == hipSuccess; ++G) {
              const int gi = gidx(f, kd, G);
              r = launch_field(f == 1, kd, G, d_til[gi], d_tiles[gi], (int)pl.tiles[gi].size(), kb,
                               koff, st);
            }
      } else if (o.time_kind == 3) {
        r = launch_update(pl.scan_upd, d_upd, d_ublocks, (int)pl.ublocks.size(), kb, koff, st);
      } else {
        r = wm_launches(o.time_kind == 2 ? 2 : 4, kb, koff);
      }
      return r == hipSuccess ? MH_OK : MH_EDEVICE;
    };
    if ((e = time_graph(c, st, o.time_k0, o.time_launches, o.time_reps, unit, o.time_us)))
      return e;
    return mark_plan_busy(c, st);
  }
  const int64_t k0 = o.k0;
  const int64_t k1 = o.k1 < 0 ? pl.kmax : o.k1;
  const bool any_res = !pl.res64.empty() || !pl.res32.empty();
  bool any_til = !pl.wm.empty() || !pl.ublocks.empty();
  // resident systems beside the tiled steps: they share no buffer but the (read-only)
  // plan, and the run's stream waits for them before the finalisation
  const bool beside = any_res && any_til && k1 > k0;
  hipStream_t rst = st;
  if (beside) {
    if (!c->side && (hipStreamCreate(&c->side) != hipSuccess ||
                     hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess ||
                     hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming) != hipSuccess))
      return MH_EDEVICE;
    if (hipEventRecord(c->fork_ev, st) != hipSuccess ||
        hipStreamWaitEvent(c->side, c->fork_ev, 0) != hipSuccess)
      return MH_EDEVICE;
    rst = c->side;
  }
  int tq = any_res && k1 > k0 ? timing_begin(c, rst, 1) : -1;
  if (launch_resident(true, pl.scan_res64, d_res64, (int)pl.res64.size(), k0, k1, pl.nmax_res64,
                      rst) != hipSuccess)
    return MH_EDEVICE;
  if (launch_resident(false, pl.scan_res32, d_res32, (int)pl.res32.size(), k0, k1, pl.nmax_res32,
                      rst) != hipSuccess)
    return MH_EDEVICE;
  timing_end(c, rst, tq);
  if (beside && hipEventRecord(c->join_ev, rst) != hipSuccess) return MH_EDEVICE;
  // the tiled steps; whatever their outcome, the run's stream then waits for the
  // resident launch (an error must not leave it reading a plan that may be re-staged)
  const int rc_til = [&]() -> int {
    // one tiled step: dipolar fields, then the per-particle update
    auto step = [&](const int64_t* kb, int64_t koff) -> int {
      int t0 = timing_begin(c, st, 0);
      for (int f = 0; f < 2; ++f)
        for (int kd = 0; kd < 2; ++kd)
          for (int G = 1; G <= 4; ++G) {
            const int gi = gidx(f, kd, G);
            if (launch_field(f == 1, kd, G, d_til[gi], d_tiles[gi], (int)pl.tiles[gi].size(), kb,
                             koff, st) != hipSuccess)
              return MH_EDEVICE;
          }
      timing_end(c, st, t0);
      t0 = timing_begin(c, st, 3);
      if (launch_update(pl.scan_upd, d_upd, d_ublocks, (int)pl.ublocks.size(), kb, koff, st) !=
          hipSuccess)
        return MH_EDEVICE;
      timing_end(c, st, t0);
      if (!pl.wm.empty()) {
        t0 = timing_begin(c, st, 2);
        if (wm_launches(2, kb, koff) != hipSuccess) return MH_EDEVICE;
        timing_end(c, st, t0);
        t0 = timing_begin(c, st, 4);
        if (wm_launches(4, kb, koff) != hipSuccess) return MH_EDEVICE;
        timing_end(c, st, t0);
      }
      return MH_OK;
    };
    int64_t k = k0;
    constexpr int64_t G = 50;
    if (any_til && c->use_graphs && !c->timing && k1 - k0 >= 2 * G) {
      if ((e = c->d_kbase.ensure(sizeof(int64_t)))) return e;
      int64_t* kb = c->d_kbase.as<int64_t>();
      // the captured kernels read the plan from d_sys at fixed offsets: reuse the graph
      // while the uploaded plan has the same layout (every pointer and count a captured
      // launch takes is part of the key)
      std::vector<uint64_t> key = {(uint64_t)(uintptr_t)c->d_sys.p, (uint64_t)off, (uint64_t)G};
      for (int gi = 0; gi < kGroups; ++gi) {
        key.push_back((uint64_t)(uintptr_t)d_til[gi]);
        key.push_back((uint64_t)(uintptr_t)d_tiles[gi]);
        key.push_back(pl.tiles[gi].size());
      }
      key.push_back((uint64_t)(uintptr_t)d_upd);
      key.push_back((uint64_t)(uintptr_t)d_ublocks);
      key.push_back(pl.ublocks.size());
      key.push_back(pl.scan_upd ? 1 : 0);
      for (auto& it : pl.wm) {
        const uint64_t* gw = reinterpret_cast<const uint64_t*>(&it.g);
        for (size_t q = 0; q < sizeof(WMArgs) / 8; ++q) key.push_back(gw[q]);
        key.push_back((uint64_t)it.first);
        key.push_back((uint64_t)it.a->R);
        key.push_back((uint64_t)it.a->p.extrema_mode);
      }
      key.push_back((uint64_t)(uintptr_t)d_wmg);
      key.push_back((uint64_t)(uintptr_t)d_wmu[0]);
      key.push_back((uint64_t)(uintptr_t)d_wmu[1]);
      key.push_back((uint64_t)pl.wmg_blocks);
      key.push_back((uint64_t)pl.wmu_blocks[0]);
      key.push_back((uint64_t)pl.wmu_blocks[1]);
      if (!c->gexec || key != c->gkey) {
        if (c->gexec) {
          (void)hipGraphExecDestroy(c->gexec);
          c->gexec = nullptr;
        }
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess)
          return MH_EDEVICE;
        int rc = MH_OK;
        for (int64_t j = 0; j < G && rc == MH_OK; ++j) rc = step(kb, j);
        if (rc == MH_OK && launch_set_step(kb, G, true, st) != hipSuccess) rc = MH_EDEVICE;
        if (hipStreamEndCapture(st, &g) != hipSuccess || rc != MH_OK) {
          if (g) (void)hipGraphDestroy(g);
          return MH_EDEVICE;
        }
        const hipError_t ie = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
          c->gexec = nullptr;
          return MH_EDEVICE;
        }
        c->gkey = key;
      }
      if (launch_set_step(kb, k0, false, st) != hipSuccess) return MH_EDEVICE;
      for (; k + G <= k1; k += G)
        if (hipGraphLaunch(c->gexec, st) != hipSuccess) return MH_EDEVICE;
    }
    for (; k < k1 && any_til; ++k)
      if ((e = step(nullptr, k))) return e;
    return MH_OK;
  }();
  if (beside && hipStreamWaitEvent(st, c->join_ev, 0) != hipSuccess) return MH_EDEVICE;
  if (rc_til) return rc_til;
  if (o.finalize) {
    if (launch_finalize(d_all, (int)all.size(), st) != hipSuccess) return MH_EDEVICE;
    for (auto& f : fin) {
      mh_asm* a = f.first;
      if (launch_finalize_asm(a->sys_area.as<double>(), (int)a->R, a->stats.as<double>(), st) !=
          hipSuccess)
        return MH_EDEVICE;
    }
  }
  if ((e = mark_plan_busy(c, st))) return e;
  for (auto& f : fin) {
    mh_asm* a = f.first;
    if (!a->done && hipEventCreateWithFlags(&a->done, hipEventDisableTiming) != hipSuccess)
      return MH_EDEVICE;
    if (hipEventRecord(a->done, st) != hipSuccess) return MH_EDEVICE;
    a->ran = true;
    a->state_parity = (int)(std::min<int64_t>(k1 - a->k_origin, total_steps(a->p)) & 1);
  }
  return MH_OK;
}

// Deterministic mean-magnetisation loops (k_master): state, accumulators and record
// only, no field buffers; replica r uses axis set r mod n_axes_sets and its amplitude.
int run_mean_loop(mh_asm* a, int64_t R, hipStream_t st) {
  mh_ctx* c = a->ctx;
  if (set_dev(c)) return MH_EDEVICE;
  if (!st) st = c->stream;
  const int64_t n = a->n;
  const int64_t rows = (int64_t)n_kept(a->p) * a->p.steps_per_period;
  int e;
  if ((e = wait_asm_idle(a))) return e;
  if ((e = a->m64.ensure(sizeof(D4) * 2 * R * n)) || (e = a->area.ensure(sizeof(double) * 2 * R * n)) ||
      (e = a->dhdip.ensure(sizeof(double) * R * n)))
    return e;
  a->resident = 0;
  a->nsplit = 1;
  a->ntiles = (int)((n + 255) / 256);
  a->rec_slots = rec_slots_for(R, a->ntiles);
  if ((e = a->recpart.ensure(sizeof(double) * R * rows * a->ntiles * a->rec_slots + 8)) ||
      (e = a->rec.ensure(sizeof(double) * R * rows + 8)) ||
      (e = a->sys_area.ensure(sizeof(double) * R)) || (e = a->stats.ensure(sizeof(double) * 4)))
    return e;
  a->R = R;
  a->seed = 0;
  a->k_origin = 0;
  std::vector<SysDesc> all;
  for (int64_t r = 0; r < R; ++r) {
    SysDesc d = make_desc(a, r);
    d.field = nullptr;
    d.field32 = nullptr;
    d.m32 = nullptr;
    all.push_back(d);
  }
  if ((e = wait_plan_free(c))) return e;  // stage reuse, whichever stream ran last
  if (hipStreamSynchronize(st) != hipSuccess) return MH_EDEVICE;
  PlanBlob blob;
  const size_t o_all = blob.put(all);
  const size_t off = blob.h.size();
  if ((e = c->h_stage.ensure(off + 256)) || (e = c->d_sys.ensure(off + 256))) return e;
  std::memcpy(c->h_stage.p, blob.h.data(), off);
  if (hipMemcpyAsync(c->d_sys.p, c->h_stage.p, off, hipMemcpyHostToDevice, st) != hipSuccess)
    return MH_EDEVICE;
  c->staged.swap(blob.h);
  SysDesc* d_all = blob_ptr<SysDesc>(c, o_all);
  if (launch_init(d_all, (int)R, (int)n, st) != hipSuccess) return MH_EDEVICE;
  const int tq = timing_begin(c, st, 5);
  if (launch_master(d_all, (int)R, (int)n, st) != hipSuccess) return MH_EDEVICE;
  timing_end(c, st, tq);
  if (launch_finalize(d_all, (int)R, st) != hipSuccess ||
      launch_finalize_asm(a->sys_area.as<double>(), (int)R, a->stats.as<double>(), st) != hipSuccess)
    return MH_EDEVICE;
  if ((e = mark_plan_busy(c, st))) return e;
  if (!a->done && hipEventCreateWithFlags(&a->done, hipEventDisableTiming) != hipSuccess)
    return MH_EDEVICE;
  if (hipEventRecord(a->done, st) != hipSuccess) return MH_EDEVICE;
  a->ran = true;
  a->state_parity = (int)(total_steps(a->p) & 1);
  return MH_OK;
}

}  // namespace


extern "C" {

int mh_run_mean_loop(mh_asm* a, int64_t n_replicas, void* hip_stream) {
  if (!a || n_replicas < 1 || n_replicas > 65535) return MH_EINVAL;
  if (a->p.interactions != 0 || !(a->p.Keff > 0) || a->p.extrema_mode != MH_EXTREMA_EXACT)
    return MH_EINVAL;
  return run_mean_loop(a, n_replicas, (hipStream_t)hip_stream);
}

// ---------------------------------------------------------------------------
// Launch-shape autotuner
// ---------------------------------------------------------------------------
namespace {

// Synthetic assembly for timing: the n nodes of a cubic lattice (spacing 1.25 d)
// nearest the centre, each moved by up to 0.1 d (so no pair overlaps), random unit
// axes; a small linear congruential generator keeps it deterministic.
void tune_geometry(int64_t n, double d, std::vector<double>& pos, std::vector<double>& axes) {
  uint64_t st = 0x9E3779B97F4A7C15ull;
  auto uni = [&]() {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(st >> 11) * 0x1.0p-53;
  };
  const int m = (int)std::ceil(std::cbrt((double)n)) + 2;
  std::vector<std::array<double, 4>> nodes;
  for (int x = -m; x <= m; ++x)
    for (int y = -m; y <= m; ++y)
      for (int z = -m; z <= m; ++z)
        nodes.push_back({(double)x, (double)y, (double)z, (double)(x * x + y * y + z * z)});
  std::stable_sort(nodes.begin(), nodes.end(),
                   [](const std::array<double, 4>& a, const std::array<double, 4>& b) {
                     return a[3] < b[3];
                   });
  pos.resize(3 * n);
  axes.resize(3 * n);
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < 3; ++c) pos[3 * i + c] = d * (1.25 * nodes[i][c] + 0.1 * (2.0 * uni() - 1.0) / std::sqrt(3.0));
    double v[3], r2 = 0.0;
    do {
      r2 = 0.0;
      for (int c = 0; c < 3; ++c) {
        v[c] = 2.0 * uni() - 1.0;
        r2 += v[c] * v[c];
      }
    } while (r2 > 1.0 || r2 < 1e-6);
    for (int c = 0; c < 3; ++c) axes[3 * i + c] = v[c] / std::sqrt(r2);
  }
}

// Seconds per time step of one run of `a` with R replicas (best of `reps`, after a
// warm-up run that absorbs allocation and graph capture).
double time_run(mh_asm* a, int64_t R, int reps) {
  mh_ctx* c = a->ctx;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
  double best = -1.0;
  for (int q = 0; q <= reps; ++q) {
    if (hipEventRecord(e0, c->stream) != hipSuccess || mh_run_loops(a, R, 12345, nullptr) ||
        hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      best = -1.0;
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    const double sec = ms * 1e-3 / (double)total_steps(a->p);
    if (q > 0 && (best < 0 || sec < best)) best = sec;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

}  // namespace

int mh_ctx_autotune(mh_ctx* c, int32_t precision, const int64_t* sizes, int32_t n_sizes,
                    const int64_t* replicas, int32_t n_replicas, const char* json_path) {
  if (!c) return MH_EINVAL;
  if (n_sizes == 0) {  // clear: back to the built-in rule
    c->shapes.clear();
    return MH_OK;
  }
  if (!sizes || n_sizes < 0 || !replicas || n_replicas < 1 || n_replicas > 64 || n_sizes > 64 ||
      (precision != MH_FP64 && precision != MH_FP32_FIELD))
    return MH_EINVAL;
  for (int q = 0; q < n_sizes; ++q)
    if (sizes[q] < 2 || sizes[q] > 200000) return MH_EINVAL;
  for (int q = 0; q < n_replicas; ++q)
    if (replicas[q] < 1 || replicas[q] > 4096) return MH_EINVAL;
  if (set_dev(c)) return MH_EDEVICE;
  mh_params p{};
  p.Ms = 4e5;
  p.Keff = 1.3e4;
  p.d = 1e-8;
  p.T = 300.0;
  p.tau0 = 1e-10;
  p.rho = 5200.0;
  p.f = 1e5;
  p.mu0Hmax = 0.02;
  p.steps_per_period = 100;
  p.n_periods = 2;
  p.n_discard = 1;
  p.prob_form = MH_P_TWO_STATE;
  p.precision = precision;
  p.interactions = 1;
  const int kinds[2] = {0, 1};
  const int bpcs[4] = {2, 3, 4, 6};
  for (int qs = 0; qs < n_sizes; ++qs) {
    std::vector<double> pos, axes;
    tune_geometry(sizes[qs], p.d, pos, axes);
    mh_asm* a = nullptr;
    int e = mh_create_assembly(c, sizes[qs], pos.data(), axes.data(), 1, &p, &a);
    if (e) return e;
    for (int qr = 0; qr < n_replicas; ++qr) {
      const int64_t R = replicas[qr];
      if (wants_resident(a, R)) continue;  // one workgroup per replica: no tile shape
      ShapeEntry best{precision == MH_FP64 ? 1 : 0, n_bucket(a->n), g_bucket(groups_of(a, R)),
                      -1, 0, 0.0};
      for (int kind : kinds)
        for (int bpc : bpcs) {
          a->force_kind = kind;
          a->force_bpc = bpc;
          const double sec = time_run(a, R, 2);
          if (sec < 0) {
            mh_destroy_assembly(a);
            return MH_EDEVICE;
          }
          if (best.tile_kind < 0 || sec * 1e6 < best.us) {
            best.tile_kind = kind;
            best.bpc = bpc;
            best.us = sec * 1e6;
          }
        }
      a->force_kind = -1;
      bool replaced = false;
      for (ShapeEntry& x : c->shapes)
        if (x.fp64 == best.fp64 && x.n_max == best.n_max && x.groups_max == best.groups_max) {
          x = best;
          replaced = true;
        }
      if (!replaced) c->shapes.push_back(best);
    }
    mh_destroy_assembly(a);
  }
  if (json_path) {
    FILE* f = std::fopen(json_path, "w");
    if (!f) return MH_EINVAL;
    std::fprintf(f, "[\n");
    for (size_t q = 0; q < c->shapes.size(); ++q) {
      const ShapeEntry& x = c->shapes[q];
      std::fprintf(f,
                   "  {\"fp64\": %d, \"n_max\": %lld, \"groups_max\": %lld, \"tile_kind\": %d, "
                   "\"blocks_per_cu\": %d, \"us_per_step\": %.3f}%s\n",
                   x.fp64, (long long)x.n_max, (long long)x.groups_max, x.tile_kind, x.bpc, x.us,
                   q + 1 < c->shapes.size() ? "," : "");
    }
    std::fprintf(f, "]\n");
    if (std::fclose(f) != 0) return MH_EINVAL;
  }
  return MH_OK;
}

int mh_ctx_load_shapes(mh_ctx* c, const char* json_path) {
  if (!c || !json_path) return MH_EINVAL;
  FILE* f = std::fopen(json_path, "r");
  if (!f) return MH_EINVAL;
  std::vector<ShapeEntry> v;
  char line[512];
  int bad = 0;
  while (std::fgets(line, sizeof(line), f)) {
    const char* b = std::strchr(line, '{');
    if (!b) continue;
    ShapeEntry x{};
    long long nm = 0, gm = 0;
    if (std::sscanf(b,
                    " {\"fp64\": %d, \"n_max\": %lld, \"groups_max\": %lld, \"tile_kind\": %d, "
                    "\"blocks_per_cu\": %d, \"us_per_step\": %lf",
                    &x.fp64, &nm, &gm, &x.tile_kind, &x.bpc, &x.us) != 6 ||
        (x.fp64 != 0 && x.fp64 != 1) || nm < 256 || gm < 1 || nm != n_bucket(nm) ||
        gm != g_bucket(gm) || (x.tile_kind != 0 && x.tile_kind != 1) || x.bpc < 1 || x.bpc > 64) {
      bad = 1;
      break;
    }
    x.n_max = nm;
    x.groups_max = gm;
    v.push_back(x);
  }
  std::fclose(f);
  if (bad || v.empty()) return MH_EINVAL;
  c->shapes = v;
  return MH_OK;
}

int mh_ctx_set_timing(mh_ctx* c, int on) {
  if (!c) return MH_EINVAL;
  if (set_dev(c)) return MH_EDEVICE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return MH_EDEVICE;
  c->timing = on ? 1 : 0;
  c->ev_used = 0;
  c->ev_kind.clear();
  return MH_OK;
}

int mh_ctx_get_timing(mh_ctx* c, int32_t kind, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return MH_EINVAL;
  if (set_dev(c)) return MH_EDEVICE;
  double tot = 0.0;
  int64_t cnt = 0;
  for (size_t q = 0; q < c->ev_kind.size(); ++q) {
    if (c->ev_kind[q] != kind) continue;
    if (hipEventSynchronize(c->ev_pool[2 * q + 1]) != hipSuccess) return MH_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_pool[2 * q], c->ev_pool[2 * q + 1]) != hipSuccess)
      return MH_EDEVICE;
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  return MH_OK;
}

const char* mh_strerror(int code) {
  switch (code) {
    case MH_OK: return "ok";
    case MH_EINVAL: return "invalid argument";
    case MH_EOVERLAP: return "particles overlap";
    case MH_ENOMEM: return "out of memory";
    case MH_EDEVICE: return "HIP device error";
    case MH_ENOTREADY: return "no finished run";
    case MH_ENUMERIC: return "non-finite value";
    case MH_EBUDGET: return "device-memory budget exceeded";
    default: return "unknown error";
  }
}

int mh_ctx_create(int device, mh_ctx** out) {
  if (!out) return MH_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MH_EDEVICE;
  mh_ctx* c = new (std::nothrow) mh_ctx();
  if (!c) return MH_ENOMEM;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess || hipStreamCreate(&c->stream) != hipSuccess) {
    delete c;
    return MH_EDEVICE;
  }
  if (hipStreamCreateWithFlags(&c->upload, hipStreamNonBlocking) != hipSuccess) {
    (void)hipStreamDestroy(c->stream);
    delete c;
    return MH_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
  if (set_resident_lds_limit() != hipSuccess || scratch_address(device, &c->scratch)) {
    (void)hipStreamDestroy(c->upload);
    (void)hipStreamDestroy(c->stream);
    delete c;
    return MH_EDEVICE;
  }
  *out = c;
  return MH_OK;
}

int mh_ctx_destroy(mh_ctx* c) {
  if (!c) return MH_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  if (c->plan_pending) (void)hipEventSynchronize(c->plan_done);
  if (c->plan_done) (void)hipEventDestroy(c->plan_done);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  for (hipGraphExec_t x : c->timing_graphs) (void)hipGraphExecDestroy(x);
  for (hipEvent_t ev : c->tev)
    if (ev) (void)hipEventDestroy(ev);
  c->d_kbase.release();
  c->d_probe.release();
  c->d_sys.release();
  c->h_stage.release();
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
    (void)hipEventDestroy(c->fork_ev);
    (void)hipEventDestroy(c->join_ev);
  }
  (void)hipStreamDestroy(c->upload);
  (void)hipStreamDestroy(c->stream);
  delete c;
  return MH_OK;
}

int mh_create_assembly_sets(mh_ctx* c, int64_t n, const double* pos, int64_t n_pos_sets,
                            const double* axes, int64_t n_axes_sets, const mh_params* params,
                            mh_asm** out) {
  if (!out) return MH_EINVAL;
  *out = nullptr;
  if (!c || !pos || !axes || n < 1 || n > (1 << 24) || n_axes_sets < 1 || n_pos_sets < 1 ||
      n_pos_sets > 65536 || n * n_pos_sets > ((int64_t)1 << 28))
    return MH_EINVAL;
  int e = validate_params(params);
  if (e) return e;
  // one interaction matrix per geometry: the matrix form takes a single position set
  if (n_pos_sets > 1 && params->precision == MH_BF16X3_WM) return MH_EINVAL;
  for (int64_t i = 0; i < 3 * n * n_pos_sets; ++i)
    if (!std::isfinite(pos[i])) return MH_EINVAL;
  std::vector<D4> ax((size_t)(n * n_axes_sets));
  for (int64_t i = 0; i < n * n_axes_sets; ++i) {
    const double x = axes[3 * i], y = axes[3 * i + 1], z = axes[3 * i + 2];
    if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z)) return MH_EINVAL;
    const double nn = std::sqrt(x * x + y * y + z * z);
    if (!(nn > 0)) return MH_EINVAL;
    ax[i] = D4{x / nn, y / nn, z / nn, 0.0};
  }
  for (int64_t q = 0; q < n_pos_sets; ++q)
    if ((e = check_overlap(n, pos + 3 * n * q, params->d))) return e;
  if (set_dev(c)) return MH_EDEVICE;
  mh_asm* a = new (std::nothrow) mh_asm();
  if (!a) return MH_ENOMEM;
  a->ctx = c;
  a->n = n;
  a->n_axes_sets = n_axes_sets;
  a->n_pos_sets = n_pos_sets;
  a->p = *params;
  const int64_t np = n * n_pos_sets;
  std::vector<D4> p64((size_t)np);
  std::vector<F4> p32((size_t)np);
  for (int64_t i = 0; i < np; ++i) {
    p64[i] = D4{pos[3 * i] / params->d, pos[3 * i + 1] / params->d, pos[3 * i + 2] / params->d, 0};
    p32[i] = F4{(float)p64[i].x, (float)p64[i].y, (float)p64[i].z, 0.f};
  }
  if ((e = a->pos64.ensure(sizeof(D4) * np)) || (e = a->pos32.ensure(sizeof(F4) * np)) ||
      (e = a->axes.ensure(sizeof(D4) * n * n_axes_sets))) {
    mh_destroy_assembly(a);
    return e;
  }
  // on the context's upload stream (the buffers are new: no earlier work touches them),
  // complete before the assembly is returned
  hipStream_t up = c->upload;
  if (hipMemcpyAsync(a->pos64.p, p64.data(), sizeof(D4) * np, hipMemcpyHostToDevice, up) !=
          hipSuccess ||
      hipMemcpyAsync(a->pos32.p, p32.data(), sizeof(F4) * np, hipMemcpyHostToDevice, up) !=
          hipSuccess ||
      hipMemcpyAsync(a->axes.p, ax.data(), sizeof(D4) * n * n_axes_sets, hipMemcpyHostToDevice,
                     up) != hipSuccess ||
      hipStreamSynchronize(up) != hipSuccess) {
    mh_destroy_assembly(a);
    return MH_EDEVICE;
  }
  *out = a;
  return MH_OK;
}

int mh_create_assembly(mh_ctx* c, int64_t n, const double* pos, const double* axes,
                       int64_t n_axes_sets, const mh_params* params, mh_asm** out) {
  return mh_create_assembly_sets(c, n, pos, 1, axes, n_axes_sets, params, out);
}

int mh_destroy_assembly(mh_asm* a) {
  if (!a) return MH_EINVAL;
  (void)hipSetDevice(a->ctx->device);
  if (a->done) {
    (void)hipEventSynchronize(a->done);
    (void)hipEventDestroy(a->done);
  }
  DevBuf* bufs[] = {&a->pos64, &a->pos32, &a->axes, &a->m64, &a->m32, &a->area, &a->dhdip, &a->recpart,
                    &a->rec, &a->sys_area, &a->stats, &a->diag, &a->tmp, &a->field,
                    &a->mhi, &a->mlo, &a->bt};
  for (auto* b : bufs) b->release();
  delete a;
  return MH_OK;
}

int mh_set_replica_fields(mh_asm* a, int64_t count, const double* mu0Hmax) {
  if (!a || count < 0 || (count > 0 && !mu0Hmax)) return MH_EINVAL;
  for (int64_t q = 0; q < count; ++q)
    if (!std::isfinite(mu0Hmax[q]) || mu0Hmax[q] < 0) return MH_EINVAL;
  a->hmax.assign(mu0Hmax, mu0Hmax + count);
  return MH_OK;
}

int mh_run_batch(mh_asm* const* asms, int32_t count, const int64_t* n_replicas,
                 const uint64_t* seeds, void* hip_stream) {
  if (!asms || count < 1 || !n_replicas || !seeds) return MH_EINVAL;
  std::vector<mh_asm*> v;
  std::vector<int64_t> R;
  std::vector<uint64_t> S;
  for (int q = 0; q < count; ++q) {
    if (!asms[q] || n_replicas[q] < 1 || n_replicas[q] > (1 << 20)) return MH_EINVAL;
    for (int w = 0; w < q; ++w)
      if (asms[w] == asms[q]) return MH_EINVAL;
    v.push_back(asms[q]);
    R.push_back(n_replicas[q]);
    S.push_back(seeds[q]);
  }
  RunOpts o;
  return run_systems(v, R, S, (hipStream_t)hip_stream, o);
}

int mh_run_loops(mh_asm* a, int64_t n_replicas, uint64_t seed, void* hip_stream) {
  mh_asm* arr[1] = {a};
  return mh_run_batch(arr, 1, &n_replicas, &seed, hip_stream);
}

int mh_time_empty_steps(mh_ctx* c, int64_t steps, double* us_per_step) {
  if (!c || !us_per_step || steps < 1 || steps > 10000000) return MH_EINVAL;
  if (set_dev(c)) return MH_EDEVICE;
  int e;
  if ((e = c->d_probe.ensure(sizeof(double)))) return e;
  if (!c->tev[0] && (hipEventCreate(&c->tev[0]) != hipSuccess || hipEventCreate(&c->tev[1]) != hipSuccess))
    return MH_EDEVICE;
  hipStream_t st = c->stream;
  float ms = 0.f;
  // one untimed launch first (code load, clocks), then the timed one
  if (launch_empty_steps(std::min<int64_t>(steps, 1000), c->d_probe.as<double>(), st) !=
          hipSuccess ||
      hipEventRecord(c->tev[0], st) != hipSuccess ||
      launch_empty_steps(steps, c->d_probe.as<double>(), st) != hipSuccess ||
      hipEventRecord(c->tev[1], st) != hipSuccess || hipEventSynchronize(c->tev[1]) != hipSuccess ||
      hipEventElapsedTime(&ms, c->tev[0], c->tev[1]) != hipSuccess)
    return MH_EDEVICE;
  *us_per_step = (double)ms * 1e3 / (double)steps;
  return MH_OK;
}

int mh_time_kernels(mh_asm* const* asms, int32_t count, int32_t kind, int32_t launches,
                    int32_t reps, double* us_per_step) {
  if (!asms || count < 1 || !us_per_step || launches < 1 || launches > 1000 || reps < 1 ||
      reps > 100000 || (kind != 0 && kind != 2 && kind != 3 && kind != 4))
    return MH_EINVAL;
  std::vector<mh_asm*> v;
  std::vector<int64_t> R;
  std::vector<uint64_t> S;
  int64_t min_steps = INT64_MAX, min_kept0 = INT64_MAX;
  for (int q = 0; q < count; ++q) {
    mh_asm* a = asms[q];
    if (!a || !a->ran || a->k_origin != 0 || a->R < 1) return MH_EINVAL;
    for (int w = 0; w < q; ++w)
      if (asms[w] == a) return MH_EINVAL;
    if (wait_asm_idle(a)) return MH_EDEVICE;
    v.push_back(a);
    R.push_back(a->R);
    S.push_back(a->seed);
    min_steps = std::min<int64_t>(min_steps, total_steps(a->p));
    min_kept0 = std::min<int64_t>(min_kept0, kept0(a->p));
  }
  RunOpts o;
  o.init = false;
  o.sync32 = false;
  o.finalize = false;
  o.time_kind = kind;
  o.time_launches = (int)std::min<int64_t>(launches, min_steps);
  // steps of the kept periods where there are enough of them (loop record and areas on)
  o.time_k0 = std::max<int64_t>(0, std::min<int64_t>(min_kept0, min_steps - o.time_launches));
  o.time_reps = reps;
  o.time_us = us_per_step;
  *us_per_step = 0.0;
  const int e = run_systems(v, R, S, v[0]->ctx->stream, o);
  if (e) return e;
  return hipStreamSynchronize(v[0]->ctx->stream) == hipSuccess ? MH_OK : MH_EDEVICE;
}

int mh_sync(mh_asm* a) {
  if (!a) return MH_EINVAL;
  if (!a->ran || !a->done) return MH_ENOTREADY;
  if (set_dev(a->ctx)) return MH_EDEVICE;
  return hipEventSynchronize(a->done) == hipSuccess ? MH_OK : MH_EDEVICE;
}

int mh_get_loop(mh_asm* a, int64_t replica, int32_t period, double* H_T, double* M_Apm) {
  if (!a || !H_T || !M_Apm) return MH_EINVAL;
  int e = mh_sync(a);
  if (e) return e;
  if (replica < 0 || replica >= a->R || period < 0 || period >= n_kept(a->p)) return MH_EINVAL;
  const int S = a->p.steps_per_period;
  const int64_t rows = (int64_t)n_kept(a->p) * S;
  if (hipMemcpy(M_Apm, a->rec.as<double>() + replica * rows + (int64_t)period * S,
                sizeof(double) * S, hipMemcpyDeviceToHost) != hipSuccess)
    return MH_EDEVICE;
  const double scale = a->p.Ms / (double)a->n;
  const double hm =
      a->hmax.empty() ? a->p.mu0Hmax : a->hmax[(size_t)(replica % (int64_t)a->hmax.size())];
  for (int k = 0; k < S; ++k) {
    M_Apm[k] *= scale;
    const int64_t kg = (int64_t)(a->p.n_discard + period) * S + k;
    H_T[k] = a->p.dt_override > 0
                 ? hm
                 : hm * std::cos(2.0 * 3.14159265358979323846 * (double)kg / (double)S);
  }
  return MH_OK;
}

int mh_get_sar(mh_asm* a, double* sar_Wkg, double* sar_se, double* area_Jm3, double* area_se,
               double* area_per_np) {
  if (!a) return MH_EINVAL;
  int e = mh_sync(a);
  if (e) return e;
  double st[2];
  if (hipMemcpy(st, a->stats.p, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
    return MH_EDEVICE;
  if (!std::isfinite(st[0]) || !std::isfinite(st[1])) return MH_ENUMERIC;
  const double conv = a->p.f / a->p.rho;
  if (sar_Wkg) *sar_Wkg = st[0] * conv;
  if (sar_se) *sar_se = st[1] * conv;
  if (area_Jm3) *area_Jm3 = st[0];
  if (area_se) *area_se = st[1];
  if (area_per_np) {
    if ((e = a->tmp.ensure(sizeof(double) * a->n))) return e;
    if (launch_area_per_np(a->area.as<double>(), (int)a->n, (int)a->R, n_kept(a->p),
                           a->tmp.as<double>(), a->ctx->stream) != hipSuccess)
      return MH_EDEVICE;
    if (hipMemcpyAsync(area_per_np, a->tmp.p, sizeof(double) * a->n, hipMemcpyDeviceToHost,
                       a->ctx->stream) != hipSuccess ||
        hipStreamSynchronize(a->ctx->stream) != hipSuccess)
      return MH_EDEVICE;
  }
  return MH_OK;
}

int mh_get_replica_areas(mh_asm* a, double* area) {
  if (!a || !area) return MH_EINVAL;
  int e = mh_sync(a);
  if (e) return e;
  return hipMemcpy(area, a->sys_area.p, sizeof(double) * a->R, hipMemcpyDeviceToHost) ==
                 hipSuccess
             ? MH_OK
             : MH_EDEVICE;
}

int mh_get_area_per_np(mh_asm* a, int64_t replica, double* area_per_np) {
  if (!a || !area_per_np) return MH_EINVAL;
  int e = mh_sync(a);
  if (e) return e;
  if (replica < 0 || replica >= a->R) return MH_EINVAL;
  if ((e = a->tmp.ensure(sizeof(double) * a->n))) return e;
  // the replica's accumulators (sum, compensation) as a one-replica set
  if (launch_area_per_np(a->area.as<double>() + replica * 2 * a->n, (int)a->n, 1, n_kept(a->p),
                         a->tmp.as<double>(), a->ctx->stream) != hipSuccess)
    return MH_EDEVICE;
  if (hipMemcpyAsync(area_per_np, a->tmp.p, sizeof(double) * a->n, hipMemcpyDeviceToHost,
                     a->ctx->stream) != hipSuccess ||
      hipStreamSynchronize(a->ctx->stream) != hipSuccess)
    return MH_EDEVICE;
  return MH_OK;
}

int mh_get_local_concentration(mh_asm* a, int32_t N, double* phi) {
  if (!a || !phi || N < 1 || N > a->n - 1) return MH_EINVAL;
  if (set_dev(a->ctx)) return MH_EDEVICE;
  int e;
  if ((e = a->tmp.ensure(sizeof(double) * a->n))) return e;
  hipStream_t st = a->ctx->stream;
  if (launch_local_conc(a->pos64.as<D4>(), (int)a->n, N, a->tmp.as<double>(), st) != hipSuccess ||
      hipMemcpyAsync(phi, a->tmp.p, sizeof(double) * a->n, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return MH_EDEVICE;
  return MH_OK;
}

int mh_get_field_error(mh_asm* a, int64_t replica, double* rel_frobenius, double* max_over_rms) {
  if (!a || !rel_frobenius || !max_over_rms) return MH_EINVAL;
  int e = mh_sync(a);
  if (e) return e;
  if (replica < 0 || replica >= a->R) return MH_EINVAL;
  const int64_t n = a->n;
  if (n < 2 || !a->p.interactions) {  // no dipolar field: nothing to approximate
    *rel_frobenius = *max_over_rms = 0.0;
    return MH_OK;
  }
  std::vector<double> m((size_t)(3 * n)), pos((size_t)(3 * n)), ax((size_t)(3 * n));
  if ((e = mh_get_moments(a, replica, m.data()))) return e;
  // the replica's geometry, back in metres, for two temporary assemblies
  std::vector<D4> p4((size_t)n);
  const int64_t pset = replica % a->n_pos_sets;
  if (hipMemcpy(p4.data(), a->pos64.as<D4>() + pset * n, sizeof(D4) * n, hipMemcpyDeviceToHost) !=
      hipSuccess)
    return MH_EDEVICE;
  for (int64_t i = 0; i < n; ++i) {
    pos[3 * i] = p4[i].x * a->p.d;
    pos[3 * i + 1] = p4[i].y * a->p.d;
    pos[3 * i + 2] = p4[i].z * a->p.d;
    ax[3 * i] = 1.0;
    ax[3 * i + 1] = ax[3 * i + 2] = 0.0;
  }
  std::vector<double> bf((size_t)(3 * n)), b64((size_t)(3 * n));
  mh_params p = a->p;
  for (int pass = 0; pass < 2; ++pass) {
    p.precision = pass == 0 ? a->p.precision : MH_FP64;
    mh_asm* t = nullptr;
    if ((e = mh_create_assembly(a->ctx, n, pos.data(), ax.data(), 1, &p, &t))) return e;
    e = mh_debug_field(t, m.data(), pass == 0 ? bf.data() : b64.data());
    mh_destroy_assembly(t);
    if (e) return e;
  }
  double num = 0.0, den = 0.0, worst = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double di = 0.0, bi = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double dd = bf[3 * i + c] - b64[3 * i + c];
      di += dd * dd;
      bi += b64[3 * i + c] * b64[3 * i + c];
    }
    num += di;
    den += bi;
    worst = std::max(worst, di);
  }
  *rel_frobenius = den > 0.0 ? std::sqrt(num / den) : 0.0;
  *max_over_rms = den > 0.0 ? std::sqrt(worst / (den / (double)n)) : 0.0;
  return MH_OK;
}

int mh_get_dhdip(mh_asm* a, int64_t replica, double* dhdip_T) {
  if (!a || !dhdip_T) return MH_EINVAL;
  int e = mh_sync(a);
  if (e) return e;
  if (replica < 0 || replica >= a->R) return MH_EINVAL;
  if (hipMemcpy(dhdip_T, a->dhdip.as<double>() + replica * a->n, sizeof(double) * a->n,
                hipMemcpyDeviceToHost) != hipSuccess)
    return MH_EDEVICE;
  const int nk = n_kept(a->p);
  for (int64_t i = 0; i < a->n; ++i) dhdip_T[i] = nk > 0 ? dhdip_T[i] / nk : 0.0;
  return MH_OK;
}

int mh_get_moments(mh_asm* a, int64_t replica, double* m) {
  if (!a || !m) return MH_EINVAL;
  int e = mh_sync(a);
  if (e) return e;
  if (replica < 0 || replica >= a->R) return MH_EINVAL;
  // the state after the last executed step lives in buffer (steps & 1)
  const int b = a->state_parity;
  std::vector<D4> h((size_t)a->n);
  if (hipMemcpy(h.data(), a->m64.as<D4>() + (int64_t)b * a->R * a->n + replica * a->n,
                sizeof(D4) * a->n, hipMemcpyDeviceToHost) != hipSuccess)
    return MH_EDEVICE;
  for (int64_t i = 0; i < a->n; ++i) {
    m[3 * i] = h[i].x;
    m[3 * i + 1] = h[i].y;
    m[3 * i + 2] = h[i].z;
  }
  return MH_OK;
}

int mh_debug_steps(mh_asm* a, int64_t n_replicas, uint64_t seed, int64_t k0, int64_t k1,
                   const double* m_in, double* diag) {
  if (!a || n_replicas < 1 || k0 < 0 || k1 < k0 || k1 > total_steps(a->p)) return MH_EINVAL;
  if (set_dev(a->ctx)) return MH_EDEVICE;
  std::vector<mh_asm*> v{a};
  std::vector<int64_t> R{n_replicas};
  std::vector<uint64_t> S{seed};
  hipStream_t st = a->ctx->stream;
  int e;
  if (!a->ran || a->R != n_replicas || a->seed != seed) {
    RunOpts o;
    o.k0 = 0;
    o.k1 = 0;
    o.finalize = false;
    if ((e = run_systems(v, R, S, st, o))) return e;
  }
  const int64_t n = a->n;
  if (m_in) {
    std::vector<D4> h((size_t)(n_replicas * n));
    for (int64_t q = 0; q < n_replicas * n; ++q) {
      const double x = m_in[3 * q], y = m_in[3 * q + 1], z = m_in[3 * q + 2];
      if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z)) return MH_EINVAL;
      h[q] = D4{x, y, z, 0.0};
    }
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(a->m64.as<D4>() + (k0 & 1) * n_replicas * n, h.data(), sizeof(D4) * h.size(),
                  hipMemcpyHostToDevice) != hipSuccess)
      return MH_EDEVICE;
  } else if (a->state_parity != (int)(k0 & 1)) {
    return MH_EINVAL;
  }
  double* d_diag = nullptr;
  if (diag) {
    if ((e = a->diag.ensure(sizeof(double) * 8 * n_replicas * n))) return e;
    d_diag = a->diag.as<double>();
  }
  RunOpts o;
  o.init = false;
  o.k0 = k0;
  o.k1 = k1;
  o.finalize = false;
  o.diag = d_diag;
  if ((e = run_systems(v, R, S, st, o))) return e;
  a->state_parity = (int)(k1 & 1);
  if (hipStreamSynchronize(st) != hipSuccess) return MH_EDEVICE;
  if (diag && hipMemcpy(diag, d_diag, sizeof(double) * 8 * n_replicas * n,
                        hipMemcpyDeviceToHost) != hipSuccess)
    return MH_EDEVICE;
  return MH_OK;
}

int mh_debug_field(mh_asm* a, const double* m, double* B_out) {
  if (!a || !m || !B_out) return MH_EINVAL;
  if (set_dev(a->ctx)) return MH_EDEVICE;
  const int64_t n = a->n;
  std::vector<mh_asm*> v{a};
  std::vector<int64_t> R{1};
  std::vector<uint64_t> S{0};
  hipStream_t st = a->ctx->stream;
  RunOpts o0;
  o0.k0 = 0;
  o0.k1 = 0;
  o0.finalize = false;
  int e;
  if ((e = run_systems(v, R, S, st, o0))) return e;
  std::vector<D4> h((size_t)n);
  for (int64_t q = 0; q < n; ++q) h[q] = D4{m[3 * q], m[3 * q + 1], m[3 * q + 2], 0.0};
  if ((e = a->diag.ensure(sizeof(double) * 8 * n))) return e;
  if (hipStreamSynchronize(st) != hipSuccess ||
      hipMemcpy(a->m64.p, h.data(), sizeof(D4) * n, hipMemcpyHostToDevice) != hipSuccess)
    return MH_EDEVICE;
  RunOpts o;
  o.init = false;
  o.k0 = 0;
  o.k1 = 1;
  o.finalize = false;
  o.field_only = true;
  o.diag = a->diag.as<double>();
  if ((e = run_systems(v, R, S, st, o))) return e;
  a->state_parity = 0;
  std::vector<double> d((size_t)(8 * n));
  if (hipStreamSynchronize(st) != hipSuccess ||
      hipMemcpy(d.data(), a->diag.p, sizeof(double) * 8 * n, hipMemcpyDeviceToHost) != hipSuccess)
    return MH_EDEVICE;
  for (int64_t q = 0; q < n; ++q)
    for (int c = 0; c < 3; ++c) B_out[3 * q + c] = d[8 * q + c];
  return MH_OK;
}

int mh_field_noalloc(mh_asm* a, const double* d_m, double* d_B, void* hip_stream) {
  if (!a || !d_m || !d_B || a->p.precision == MH_BF16X3_WM) return MH_EINVAL;
  mh_ctx* c = a->ctx;
  if (!c->scratch) return MH_EDEVICE;
  if (set_dev(c)) return MH_EDEVICE;
  hipStream_t st = hip_stream ? (hipStream_t)hip_stream : c->stream;
  // the launch form mh_debug_field takes (one replica), so the sums run in its order
  const int64_t n = a->n;
  const bool fp64 = a->p.precision == MH_FP64;
  const bool resident = wants_resident(a, 1);
  const int kind = tile_kind_for(a, 1);
  const int nsplit = resident ? 1 : nsplit_for(a, 1, kind);
  const int ntiles = resident ? 1 : (int)((n + 255) / 256);
  const int tpp = (int)((n + tile_width(kind) - 1) / tile_width(kind));
  const int parts = a->p.interactions ? nsplit : 0;  // no field tiles without Eq. 1
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) & ~(size_t)255;
    return o;
  };
  const size_t o_desc = take(sizeof(SysDesc));
  const size_t o_tiles = take(sizeof(int4) * (size_t)tpp * nsplit);
  const size_t o_ub = take(sizeof(int2) * (size_t)ntiles);
  const size_t o_m64 = take(sizeof(D4) * (size_t)n);
  const size_t o_m32 = fp64 ? 0 : take(sizeof(F4) * (size_t)n);
  const size_t o_field =
      resident ? 0 : take((fp64 ? sizeof(D4) : sizeof(F4)) * (size_t)n * nsplit);
  const size_t o_diag = take(sizeof(double) * 8 * (size_t)n);
  if (off > kNoAllocBytes) return MH_EBUDGET;
  unsigned char* b = c->scratch;
  SysDesc s = desc_physics(a, 0);
  s.m64 = reinterpret_cast<D4*>(b + o_m64);
  s.m32 = fp64 ? nullptr : reinterpret_cast<F4*>(b + o_m32);
  s.field = resident || !fp64 ? nullptr : reinterpret_cast<D4*>(b + o_field);
  s.field32 = resident || fp64 ? nullptr : reinterpret_cast<F4*>(b + o_field);
  s.diag = reinterpret_cast<double*>(b + o_diag);
  s.nsplit = parts;
  s.ntiles = ntiles;
  s.rec_slots = rec_slots_for(1, ntiles);
  s.stride = n;
  s.field_only = 1;
  SysDesc* d_desc = reinterpret_cast<SysDesc*>(b + o_desc);
  int4* d_tiles = reinterpret_cast<int4*>(b + o_tiles);
  int2* d_ub = reinterpret_cast<int2*>(b + o_ub);
  const bool scan = a->p.extrema_mode == MH_EXTREMA_SCAN200;
  if (launch_field_plan(s, d_desc, d_tiles, tpp, parts, d_ub, ntiles, d_m, st) != hipSuccess)
    return MH_EDEVICE;
  if (resident) {
    if (launch_resident(fp64, scan, d_desc, 1, 0, 1, (int)n, st) != hipSuccess) return MH_EDEVICE;
  } else if (launch_field(fp64, kind, 1, d_desc, d_tiles, tpp * parts, nullptr, 0, st) !=
                 hipSuccess ||
             launch_update(scan, d_desc, d_ub, ntiles, nullptr, 0, st) != hipSuccess) {
    return MH_EDEVICE;
  }
  return launch_field_out(s.diag, d_B, (int)n, st) == hipSuccess ? MH_OK : MH_EDEVICE;
}

int mh_debug_philox(mh_ctx* c, uint64_t seed, uint64_t stream, int64_t n_blocks,
                    const uint64_t* ctr, uint64_t* out) {
  if (!c || !ctr || !out || n_blocks < 1 || n_blocks > (1 << 26)) return MH_EINVAL;
  if (set_dev(c)) return MH_EDEVICE;
  void *dc = nullptr, *dout = nullptr;
  const size_t bytes = sizeof(uint64_t) * 4 * n_blocks;
  int rc = MH_OK;
  if (hipMalloc(&dc, bytes) != hipSuccess || hipMalloc(&dout, bytes) != hipSuccess) {
    rc = MH_ENOMEM;
  } else if (hipMemcpy(dc, ctr, bytes, hipMemcpyHostToDevice) != hipSuccess ||
             launch_philox_raw(seed, stream, (const uint64_t*)dc, (uint64_t*)dout, n_blocks,
                               c->stream) != hipSuccess ||
             hipStreamSynchronize(c->stream) != hipSuccess ||
             hipMemcpy(out, dout, bytes, hipMemcpyDeviceToHost) != hipSuccess) {
    rc = MH_EDEVICE;
  }
  if (dc) (void)hipFree(dc);
  if (dout) (void)hipFree(dout);
  return rc;
}

int mh_debug_sw(mh_ctx* c, int64_t n, const double* hx, const double* hy, const double* theta0,
                double* out) {
  return mh_debug_sw_mode(c, MH_EXTREMA_EXACT, n, hx, hy, theta0, out);
}

int mh_debug_sw_mode(mh_ctx* c, int32_t extrema_mode, int64_t n, const double* hx,
                     const double* hy, const double* theta0, double* out) {
  if (!c || !hx || !hy || !theta0 || !out || n < 1 || n > (1 << 26)) return MH_EINVAL;
  if (extrema_mode != MH_EXTREMA_EXACT && extrema_mode != MH_EXTREMA_SCAN200) return MH_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(hx[i]) || !std::isfinite(hy[i]) || !(hy[i] >= 0) ||
        !(std::fabs(theta0[i]) <= 3.14159265358979323846))
      return MH_EINVAL;
  if (set_dev(c)) return MH_EDEVICE;
  double* d = nullptr;
  const size_t in = sizeof(double) * n;
  int rc = MH_OK;
  if (hipMalloc(&d, in * 9) != hipSuccess) return MH_ENOMEM;
  if (hipMemcpy(d, hx, in, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d + n, hy, in, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d + 2 * n, theta0, in, hipMemcpyHostToDevice) != hipSuccess ||
      launch_sw(d, d + n, d + 2 * n, d + 3 * n, n, extrema_mode == MH_EXTREMA_SCAN200,
                c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess ||
      hipMemcpy(out, d + 3 * n, in * 6, hipMemcpyDeviceToHost) != hipSuccess)
    rc = MH_EDEVICE;
  (void)hipFree(d);
  return rc;
}

}  // extern "C"

// ===========================================================================
// Continuous-batching server
//
// A scheduler thread keeps one global step clock. Every iteration it admits queued
// requests in arrival order while their device memory fits the budget, then advances
// every admitted request by one chunk of steps in a single fused launch sequence
// (requests at different points of their runs share the launches; each reads its own
// local step = clock - origin). A request runs in rounds of up to 64 replicas on
// consecutive Philox streams; after each round the replica areas are appended on the
// device and reduced, and the request finishes once 2 SE <= max(target |A|, floor)
// with at least min_replicas, or at max_replicas. Its result depends only on its own
// inputs: launch forms are chosen per assembly and every system has its own streams.
// ===========================================================================
namespace {

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct SReq {
  uint64_t id = 0;
  mh_asm* a = nullptr;
  uint64_t seed = 0;
  double target = 0.01;
  double floor = 0.0;  // absolute floor of 2 SE (J/m^3)
  int64_t minR = 64, maxR = 8192, done_R = 0, round_R = 0;
  int state = 0;  // 0 queued, 1 running, 2 done
  int64_t end = 0;
  size_t bytes = 0;
  DevBuf areas;  // per-replica areas of finished rounds
  mh_result res{};
  std::atomic<int64_t> progress{0};  // replicas of finished rounds, for polls in flight
};

// Device memory a request holds while admitted: its geometry and the buffers that
// prepare_run allocates for rounds of R replicas, under the launch form (resident,
// tile shape and source parts) its runs will take, plus the per-replica areas of up to
// maxR replicas.
size_t request_bytes(const mh_asm* a, int64_t R, int64_t maxR) {
  const mh_params& p = a->p;
  const int64_t n = a->n;
  const bool resident = wants_resident(a, R);
  const bool wm = p.precision == MH_BF16X3_WM;
  const int64_t rows = (int64_t)n_kept(p) * p.steps_per_period;
  const int64_t ntiles = resident ? 1 : (n + 255) / 256;
  const int64_t nsplit = resident ? 1 : nsplit_for(a, R, tile_kind_for(a, R));
  size_t b = (size_t)n * a->n_pos_sets * (sizeof(D4) + sizeof(F4)) +
             (size_t)n * a->n_axes_sets * sizeof(D4);
  b += (size_t)R * n * (2 * sizeof(D4) + 2 * sizeof(double) + sizeof(double));
  if (p.precision == MH_FP32_FIELD) b += (size_t)R * n * 2 * sizeof(F4);
  b += sizeof(double) * ((size_t)R * rows * ntiles * rec_slots_for(R, ntiles) + 8);
  b += sizeof(double) * ((size_t)R * rows + 8) + sizeof(double) * (R + 4);
  if (!resident && !wm)
    b += (p.precision == MH_FP32_FIELD ? sizeof(F4) : sizeof(D4)) * (size_t)R * n * nsplit;
  if (wm) {
    const int64_t rq = 8 * wm_tile_rows(), kq = wm_tile_k();
    const int64_t Mp = (3 * n + rq - 1) / rq * rq, Kp = (3 * n + kq - 1) / kq * kq;
    const int64_t Rp = (R + wm_tile_reps() - 1) / wm_tile_reps() * wm_tile_reps();
    b += 2 * sizeof(__bf16) * (size_t)Rp * Kp + sizeof(float) * (size_t)wm_ksplit() * Rp * Mp;
  }
  return b + sizeof(double) * (size_t)maxR;
}

}  // namespace

struct mh_server {
  mh_ctx* ctx = nullptr;
  size_t budget = 0, used = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<SReq*> queue;
  std::vector<SReq*> running;
  std::unordered_map<uint64_t, SReq*> reqs;
  uint64_t next_id = 1;
  bool stop = false;
  int64_t clock = 0;
  int chunk = 100;  // steps per scheduling chunk: two replays of the 50-step graph
  int64_t round_size = 64;
  int error = 0;
  std::thread th;
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};  // end of the last two enqueued chunks
  int64_t chunk_no = 0;
  void loop();
  int start_round(SReq* q);
  int finish_round(SReq* q, bool& done);
};

int mh_server::start_round(SReq* q) {
  // the matrix form pads replicas to 256 per product, so it runs rounds of 256
  const int64_t rs = q->a->p.precision == MH_BF16X3_WM ? 4 * round_size : round_size;
  q->round_R = std::min<int64_t>(rs, q->maxR - q->done_R);
  q->a->k_origin = clock;
  q->a->stream_base = (uint64_t)q->done_R;
  std::vector<mh_asm*> v{q->a};
  std::vector<int64_t> R{q->round_R};
  std::vector<uint64_t> S{q->seed};
  RunOpts o;
  o.k0 = o.k1 = clock;
  o.finalize = false;
  const int e = run_systems(v, R, S, ctx->stream, o);
  q->end = clock + total_steps(q->a->p);
  q->state = 1;
  return e;
}

int mh_server::finish_round(SReq* q, bool& done) {
  std::vector<mh_asm*> v{q->a};
  std::vector<int64_t> R{q->round_R};
  std::vector<uint64_t> S{q->seed};
  RunOpts o;
  o.init = false;
  o.sync32 = false;
  o.k0 = o.k1 = clock;
  int e = run_systems(v, R, S, ctx->stream, o);
  if (e) return e;
  hipStream_t st = ctx->stream;
  if (hipMemcpyAsync(q->areas.as<double>() + q->done_R, q->a->sys_area.p,
                     sizeof(double) * q->round_R, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return MH_EDEVICE;
  q->done_R += q->round_R;
  q->progress.store(q->done_R, std::memory_order_relaxed);
  if (launch_finalize_asm(q->areas.as<double>(), (int)q->done_R, q->a->stats.as<double>(), st) !=
      hipSuccess)
    return MH_EDEVICE;
  double stt[2];
  if (hipMemcpyAsync(stt, q->a->stats.p, sizeof(stt), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return MH_EDEVICE;
  const mh_params& p = q->a->p;
  const bool conv =
      q->done_R >= q->minR && 2.0 * stt[1] <= std::max(q->target * std::fabs(stt[0]), q->floor);
  done = conv || q->done_R >= q->maxR;
  if (done) {
    q->res.area_Jm3 = stt[0];
    q->res.area_se = stt[1];
    q->res.sar_Wkg = stt[0] * p.f / p.rho;
    q->res.sar_se = stt[1] * p.f / p.rho;
    q->res.replicas = q->done_R;
    q->res.loops = q->done_R * (p.n_periods - p.n_discard);
    q->res.done_ns = now_ns();
    q->res.status = std::isfinite(stt[0]) ? MH_OK : MH_ENUMERIC;
  }
  return MH_OK;
}

void mh_server::loop() {
  if (set_dev(ctx)) {
    error = MH_EDEVICE;
    return;
  }
  for (;;) {
    std::vector<SReq*> admit;
    {
      std::unique_lock<std::mutex> lk(mu);
      while (!stop && queue.empty() && running.empty()) cv.wait(lk);
      if (stop && running.empty() && queue.empty()) break;
      if (stop) {  // drop queued work on shutdown
        for (auto* q : queue) q->state = 2, q->res.status = MH_EINVAL;
        queue.clear();
      }
      while (!queue.empty() && used + queue.front()->bytes <= budget) {
        SReq* q = queue.front();
        queue.pop_front();
        used += q->bytes;
        admit.push_back(q);
      }
    }
    for (auto* q : admit) {
      q->res.start_ns = now_ns();
      int e = q->areas.ensure(sizeof(double) * q->maxR);
      if (!e) e = start_round(q);
      if (e) {
        std::lock_guard<std::mutex> lk(mu);
        q->state = 2;
        q->res.status = e;
        q->res.done_ns = now_ns();
        used -= q->bytes;
        continue;
      }
      running.push_back(q);
    }
    if (running.empty()) continue;
    // one chunk of steps for every running request
    std::vector<mh_asm*> v;
    std::vector<int64_t> R;
    std::vector<uint64_t> S;
    for (auto* q : running) {
      v.push_back(q->a);
      R.push_back(q->round_R);
      S.push_back(q->seed);
    }
    RunOpts o;
    o.init = false;
    o.sync32 = false;
    o.finalize = false;
    o.k0 = clock;
    o.k1 = clock + chunk;
    // bounded run-ahead: the host enqueues a chunk only once the chunk before the
    // previous one has finished, so a request admitted now starts within about two
    // chunks instead of behind a long queue of enqueued ones
    int e = MH_OK;
    hipEvent_t& ev = chunk_ev[chunk_no & 1];
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) e = MH_EDEVICE;
    if (!e && chunk_no >= 2 && hipEventSynchronize(ev) != hipSuccess) e = MH_EDEVICE;
    if (!e) e = run_systems(v, R, S, ctx->stream, o);
    if (!e && hipEventRecord(ev, ctx->stream) != hipSuccess) e = MH_EDEVICE;
    ++chunk_no;
    clock += chunk;
    std::vector<SReq*> still;
    for (auto* q : running) {
      bool done = false;
      if (!e && q->end <= clock) {
        int e2 = finish_round(q, done);
        if (!e2 && !done) e2 = start_round(q);
        if (e2) {
          done = true;
          q->res.status = e2;
          q->res.done_ns = now_ns();
        }
      } else if (e) {
        done = true;
        q->res.status = e;
        q->res.done_ns = now_ns();
      }
      if (done) {
        mh_destroy_assembly(q->a);
        q->a = nullptr;
        q->areas.release();
        std::lock_guard<std::mutex> lk(mu);
        q->state = 2;
        used -= q->bytes;
      } else {
        still.push_back(q);
      }
    }
    running.swap(still);
  }
}

extern "C" {

int mh_server_create(mh_ctx* ctx, size_t hbm_budget_bytes, mh_server** out) {
  if (!ctx || !out || hbm_budget_bytes == 0) return MH_EINVAL;
  mh_server* s = new (std::nothrow) mh_server();
  if (!s) return MH_ENOMEM;
  // a private context: the scheduler's stream, plan buffers and graphs are its own
  int e = mh_ctx_create(ctx->device, &s->ctx);
  if (e) {
    delete s;
    return e;
  }
  s->budget = hbm_budget_bytes;
  s->ctx->shapes = ctx->shapes;  // requests run with the launch shapes of the caller's context
  s->th = std::thread([s] { s->loop(); });
  *out = s;
  return MH_OK;
}

int mh_server_submit(mh_server* s, const mh_request* rq, uint64_t* req_id) {
  if (!s || !rq || !req_id) return MH_EINVAL;
  if (rq->min_replicas < 1 || rq->max_replicas < rq->min_replicas || rq->max_replicas > (1 << 20) ||
      !(rq->target_rel_err > 0))
    return MH_EINVAL;
  if (!std::isfinite(rq->abs_err_floor) || rq->abs_err_floor < 0) return MH_EINVAL;
  const int64_t rs = rq->params.precision == MH_BF16X3_WM ? 4 * s->round_size : s->round_size;
  const int64_t R = std::min<int64_t>(rs, rq->max_replicas);
  mh_asm* a = nullptr;
  int e = mh_create_assembly(s->ctx, rq->n, rq->pos, rq->axes, rq->n_axes_sets, &rq->params, &a);
  if (e) return e;
  const size_t bytes = request_bytes(a, R, rq->max_replicas);
  if (bytes > s->budget) {
    mh_destroy_assembly(a);
    return MH_EBUDGET;
  }
  SReq* q = new (std::nothrow) SReq();
  if (!q) {
    mh_destroy_assembly(a);
    return MH_ENOMEM;
  }
  q->a = a;
  q->seed = rq->seed;
  q->target = rq->target_rel_err;
  q->floor = rq->abs_err_floor;
  q->minR = rq->min_replicas;
  q->maxR = rq->max_replicas;
  q->bytes = bytes;
  q->res.submit_ns = now_ns();
  q->res.status = MH_ENOTREADY;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      mh_destroy_assembly(a);
      delete q;
      return MH_EINVAL;
    }
    q->id = s->next_id++;
    s->reqs[q->id] = q;
    s->queue.push_back(q);
  }
  s->cv.notify_one();
  *req_id = q->id;
  return MH_OK;
}

int mh_server_poll(mh_server* s, uint64_t req_id, mh_result* out) {
  if (!s || !out) return MH_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(req_id);
  if (it == s->reqs.end()) return MH_EINVAL;
  if (it->second->state != 2) {
    // progress so far: replicas of the rounds finished, no result yet
    *out = mh_result{};
    out->replicas = it->second->progress.load(std::memory_order_relaxed);
    out->submit_ns = it->second->res.submit_ns;
    out->start_ns = it->second->res.start_ns;
    out->status = MH_ENOTREADY;
    return MH_ENOTREADY;
  }
  *out = it->second->res;
  return MH_OK;
}

int mh_server_destroy(mh_server* s) {
  if (!s) return MH_EINVAL;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_one();
  if (s->th.joinable()) s->th.join();
  for (auto& kv : s->reqs) {
    if (kv.second->a) mh_destroy_assembly(kv.second->a);
    delete kv.second;
  }
  for (hipEvent_t ev : s->chunk_ev)
    if (ev) (void)hipEventDestroy(ev);
  mh_ctx_destroy(s->ctx);
  delete s;
  return MH_OK;
}

}  // extern "C"
