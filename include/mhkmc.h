/*
 * mhkmc: kinetic Monte-Carlo hysteresis loops of interacting magnetic nanoparticles
 * on one AMD Instinct MI355X (gfx950).
 *
 * Method: R. P. Tan, J. Carrey and M. Respaud, "Magnetic hyperthermia properties of
 * nanoparticles inside lysosomes using kinetic Monte-Carlo simulations", arXiv:1407.2737.
 * Each time step of a sinusoidal applied field (Sec. II.1, steps i-viii):
 *   - the exact dipolar field on every particle from all others (Eq. 1),
 *   - the Stoner-Wohlfarth minima and lower maximum of Eq. 2 in the particle's
 *     working plane, and the fall of the moment into its basin (steps iii-v),
 *   - the two-state switching probability of Eqs. 3-5 and a uniform draw (vi-vii),
 *   - accumulation of the loop and of its area; SAR = A f / rho (Sec. III.2.a).
 * All particles move synchronously from the start-of-step state (Sec. II.2).
 *
 * Conventions
 *   - SI units throughout: positions in m, M_S in A/m, K_eff in J/m^3, mu0 H in T,
 *     areas in J/m^3, SAR in W/kg.
 *   - Every function returns 0 on success or a negative MH_E* code; no exception or
 *     abort crosses this boundary. mh_strerror() names a code.
 *   - Input arrays are host memory, read during the call and copied; the caller keeps
 *     ownership. Output arrays are host memory of the documented size, allocated by
 *     the caller. The library owns all device memory it allocates until the matching
 *     destroy call.
 *   - One assembly must not be driven from two threads at once.
 */
#ifndef MHKMC_H
#define MHKMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define MH_OK 0
#define MH_EINVAL -1     /* invalid argument (null pointer, bad size, non-finite value) */
#define MH_EOVERLAP -2   /* two particles closer than one diameter */
#define MH_ENOMEM -3     /* device or host allocation failed */
#define MH_EDEVICE -4    /* HIP runtime error (no device, launch failure) */
#define MH_ENOTREADY -5  /* results requested before a run finished */
#define MH_ENUMERIC -6   /* non-finite value produced during a run */
#define MH_EBUDGET -7    /* request exceeds the configured device-memory budget */

/* precision of the dipolar sum (the per-particle barrier step is always FP64) */
#define MH_FP64 0        /* Eq. 1 summed in FP64 */
#define MH_FP32_FIELD 1  /* Eq. 1 summed in FP32 from FP32 positions / d */
#define MH_BF16X3_WM 2   /* fixed interaction matrix W (3N x 3N) times moments on MFMA,
                            BF16 hi+lo split, FP32 accumulation */

/* probability of leaving the current well during one step */
#define MH_P_TWO_STATE 0   /* Eq. 5: nu_c/(nu_c+nu_o) (1 - exp(-(nu_c+nu_o) dt)) */
#define MH_P_SINGLE_RATE 1 /* 1 - exp(-nu_c dt): the one-rate limit of Eq. 5 */

/* search for the energy extrema of one particle in its working plane (Sec. II.1, step iv) */
#define MH_EXTREMA_EXACT 0   /* every stationary point of Eq. 2, found by sign-change
                                brackets and Newton polish in direction form; the two
                                minima are present exactly when the field lies inside
                                the Stoner-Wohlfarth astroid */
#define MH_EXTREMA_SCAN200 1 /* the paper's search taken literally: dE/dtheta sampled on
                                200 angles 2 pi j/200, each sign change refined by Newton's
                                method from its interval's midpoint (at most 50 steps, until
                                a step is below 1e-13). Within about 1e-4 of the switching
                                field a saddle and the minimum beside it can share one grid
                                interval and are then missed: the particle switches that
                                much early. FP64 sin/cos per grid point, so several times
                                slower per particle step than MH_EXTREMA_EXACT */

typedef struct mh_ctx mh_ctx;
typedef struct mh_asm mh_asm;

/* Material, field and protocol of one assembly (Sec. II.1, Sec. II.2 defaults). */
typedef struct {
  double Ms;          /* saturation magnetisation, A/m (> 0) */
  double Keff;        /* uniaxial anisotropy, J/m^3 (>= 0; 0 = moments follow the field) */
  double d;           /* particle diameter, m (> 0); V = pi d^3 / 6 */
  double T;           /* temperature, K (>= 0; 0 = no thermal jumps, step vii skipped) */
  double tau0;        /* inverse attempt frequency 1/nu0, s (> 0; paper: 1e-10) */
  double rho;         /* density for SAR, kg/m^3 (> 0; paper: 5200) */
  double f;           /* field frequency, Hz (> 0) */
  double mu0Hmax;     /* field amplitude, T (>= 0); H_k = Hmax cos(2 pi k/S) e_H */
  double dt_override; /* > 0: constant field mu0Hmax e_H and steps of this length, s */
  double field_dir[3];/* direction of the applied field, normalised to e_H; (0, 0, 0) means
                         +x, the paper's choice (Sec. II.1). Moments start as
                         sign(n . e_H) n; loops (mh_get_loop), areas, SAR and Eq. 6
                         (mh_get_dhdip) use the components along e_H */
  int32_t steps_per_period; /* S, even, >= 2 (paper: 2000) */
  int32_t n_periods;        /* periods run (>= 1) */
  int32_t n_discard;        /* leading periods not kept (0 <= n_discard < n_periods) */
  int32_t prob_form;        /* MH_P_TWO_STATE or MH_P_SINGLE_RATE */
  int32_t precision;        /* MH_FP64, MH_FP32_FIELD or MH_BF16X3_WM */
  int32_t interactions;     /* 1: Eq. 1 on; 0: off (the paper's validation mode, Sec. II.3) */
  int32_t extrema_mode;     /* MH_EXTREMA_EXACT or MH_EXTREMA_SCAN200 */
  int32_t reserved;         /* must be 0 */
} mh_params;

/* Context bound to one HIP device; owns a default stream. */
int mh_ctx_create(int device, mh_ctx** out);
int mh_ctx_destroy(mh_ctx* ctx);

/* Assembly of n particles (Sec. II.1).
 *   pos   n x 3 row-major centres, m. Pairs closer than d (1 - 1e-9) are rejected
 *         with MH_EOVERLAP.
 *   axes  n_axes_sets x n x 3 easy axes (normalised on input, zero rows rejected).
 *         Replica r uses axis set r mod n_axes_sets: one set shared by all replicas,
 *         or one per replica (averaging over axis orientations, Sec. III.1).
 * Initial moments are m_i = sign(n_i . e_H) n_i (sign(0) = +1), e_H the unit field
 * direction of params.field_dir. */
int mh_create_assembly(mh_ctx* ctx, int64_t n, const double* pos, const double* axes,
                       int64_t n_axes_sets, const mh_params* params, mh_asm** out);

/* As mh_create_assembly with n_pos_sets position sets (pos: n_pos_sets x n x 3, each
 * set checked for overlaps): replica r uses position set r mod n_pos_sets, the
 * paper's second averaging method (Sec. III.1), in which positions as well as axes
 * change between loops and particle i of every set sits near the same mean position
 * (for instance the same lattice node). Per-particle outputs therefore refer to that
 * mean position. The interaction-matrix form holds one matrix per geometry and takes
 * a single set (MH_EINVAL otherwise); mh_get_local_concentration and mh_debug_field use
 * set 0. */
int mh_create_assembly_sets(mh_ctx* ctx, int64_t n, const double* pos, int64_t n_pos_sets,
                            const double* axes, int64_t n_axes_sets, const mh_params* params,
                            mh_asm** out);
int mh_destroy_assembly(mh_asm* a);

/* Runs n_periods x steps_per_period steps for n_replicas independent replicas.
 * Replica r draws its uniforms from Philox-4x64-10 with key (seed, r) and counter
 * (i/4, k, 0, 0), word i mod 4, u = (word >> 11) 2^-53; it jumps iff u < P.
 * hip_stream: a hipStream_t, or NULL for the context's stream. Asynchronous with
 * respect to the host; results are read after mh_sync. */
int mh_run_loops(mh_asm* a, int64_t n_replicas, uint64_t seed, void* hip_stream);

/* Per-replica field amplitudes for later runs: replica r uses mu0Hmax[r mod count]
 * (T) instead of params.mu0Hmax, e.g. an amplitude sweep on one lysosome
 * (Sec. III.2.b). count = 0 restores params.mu0Hmax. */
int mh_set_replica_fields(mh_asm* a, int64_t count, const double* mu0Hmax);

/* Runs several assemblies together (uneven sizes, different materials and fields):
 * one fused launch per step covers every assembly that still has steps to run, and
 * small assemblies run all their steps inside one launch. Each assembly's results are
 * those it would give alone with the same (n_replicas, seed). */
int mh_run_batch(mh_asm* const* asms, int32_t count, const int64_t* n_replicas,
                 const uint64_t* seeds, void* hip_stream);

/* Deterministic mean-magnetisation loops of non-interacting particles: the paper's
 * validation method (Sec. II.3, Fig. 1(c)-(d)), the loop of an infinite number of
 * particles. Instead of drawing one well per particle, each particle carries the
 * probability of each well; every step both weighted moments fall in the applied field
 * (steps iii-v), weights reaching the same minimum are pooled, and Eq. 5 moves weight
 * across the barrier in both directions (steps vi-vii). Replica r uses axis set
 * r mod n_axes_sets and, after mh_set_replica_fields, its own amplitude; no random
 * numbers are drawn. Results are read with mh_get_loop, mh_get_sar,
 * mh_get_replica_areas and mh_get_area_per_np as after mh_run_loops; mh_get_moments
 * gives the expected moments. Asynchronous like mh_run_loops (hip_stream NULL = the
 * library's stream). MH_EINVAL unless params.interactions == 0, Keff > 0 and
 * extrema_mode == MH_EXTREMA_EXACT, or for n_replicas outside [1, 65535]. */
int mh_run_mean_loop(mh_asm* a, int64_t n_replicas, void* hip_stream);

/* Waits for the assembly's last run. */
int mh_sync(mh_asm* a);

/* Loop of one replica for kept period p (0 <= p < n_periods - n_discard):
 *   H_T[k]   applied mu0 H_k (T), k = 0 .. S-1
 *   M_Apm[k] M_S <m . e_H> after step k (A/m), the magnetisation along the field. */
int mh_get_loop(mh_asm* a, int64_t replica, int32_t period, double* H_T, double* M_Apm);

/* Loop area A (J/m^3: mean over particles and kept periods, averaged over replicas)
 * with its standard error over replicas, SAR = A f / rho (W/kg) and its standard error.
 * area_per_np: n replica-mean per-particle areas, or NULL. */
int mh_get_sar(mh_asm* a, double* sar_Wkg, double* sar_se, double* area_Jm3, double* area_se,
               double* area_per_np);

/* Per-replica loop areas (n_replicas values, J/m^3). */
int mh_get_replica_areas(mh_asm* a, double* area);

/* Per-particle loop areas of one replica (n values, J/m^3, mean over its kept periods):
 * the energy each particle absorbs, Sec. II.2 area rule applied to one moment, which
 * the per-particle analyses of Sec. III (area against depth below the lysosome
 * membrane) average. MH_EINVAL for a replica outside the last run, MH_ENOTREADY before
 * any run. */
int mh_get_area_per_np(mh_asm* a, int64_t replica, double* area_per_np);

/* Error of the assembly's field form on one replica's current moments: the Eq. 1 field
 * computed by the assembly's precision (FP32 sums or the BF16x3 matrix product) against
 * the FP64 kernel, as the relative Frobenius norm over all particles and components and
 * as the largest per-particle error over the rms field. Computed on temporary copies of
 * the geometry; the assembly's run and results are left as they are. 0 for FP64, without
 * interactions or for one particle. Synchronous; MH_EINVAL for a replica outside the
 * last run, MH_ENOTREADY before any run. */
int mh_get_field_error(mh_asm* a, int64_t replica, double* rel_frobenius, double* max_over_rms);

/* Eq. 6 per particle of one replica (n values, tesla): the e_H component of the dipolar
 * field acting in the +mu0 Hmax step (k = 0 mod S, from that step's start-of-step
 * moments) minus that in the -mu0 Hmax step (k = S/2 mod S), averaged over the kept
 * periods; positive where the neighbours' field reinforces the applied one (Sec.
 * III.3). Zero without interactions and after mh_run_mean_loop. MH_EINVAL for a
 * replica outside the last run, MH_ENOTREADY before any run. */
int mh_get_dhdip(mh_asm* a, int64_t replica, double* dhdip_T);

/* Local volume concentration of Eq. 8 (Sec. III.5) for every particle (n values):
 * phi_N = 3 N V / (4 pi r_N^3) = N d^3 / (8 r_N^3), with r_N the exact distance to the
 * particle's N-th nearest neighbour. Geometry only (no run needed); synchronous.
 * MH_EINVAL unless 1 <= N <= n - 1. */
int mh_get_local_concentration(mh_asm* a, int32_t N, double* phi);

/* Current moments of one replica (n x 3). */
int mh_get_moments(mh_asm* a, int64_t replica, double* m);

/* Diagnostics for kernel-level parity. Run steps [k0, k1) of replica set
 * (n_replicas, seed) starting from moments m_in (n_replicas x n x 3, or NULL to keep
 * the current state), without resetting the area accumulators. When diag is not NULL
 * the last step writes, per replica and particle, 8 doubles: total field B (3, T),
 * switching probability P, jump flag, two-minima flag, 0, 0. */
int mh_debug_steps(mh_asm* a, int64_t n_replicas, uint64_t seed, int64_t k0, int64_t k1,
                   const double* m_in, double* diag);

/* Allocation-free form of mh_debug_field, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 *   d_m  device pointer, n x 3 doubles (row-major): the moments, read during the call's
 *        work on the stream.
 *   d_B  device pointer, n x 3 doubles: receives the Eq. 1 field (T) summed exactly as
 *        mh_debug_field sums it (same kernels, launch form and order: bitwise the same
 *        result). Both buffers stay the caller's.
 *   hip_stream  a hipStream_t, or NULL for the context's stream. The call only enqueues
 *        kernels (no allocation, no copy from the host, no synchronisation); d_B holds the
 *        field once the stream has reached it, so it may be captured into a HIP graph.
 * Every intermediate (descriptor, tile lists, moment copies, partial sums) lives in one
 * fixed 16 MiB device array per GPU, owned by the library for the life of the process
 * and shared by all calls on that GPU: enough for about 100 000 particles under the
 * built-in launch shapes. Calls that overlap on one GPU (other streams, other threads)
 * race on it; serialise them. The assembly's run state and results are not touched.
 * MH_EINVAL for a null pointer or an interaction-matrix (MH_BF16X3_WM) assembly,
 * MH_EBUDGET when the evaluation needs more than the fixed array, MH_EDEVICE for a
 * launch failure. */
int mh_field_noalloc(mh_asm* a, const double* d_m, double* d_B, void* hip_stream);

/* Raw Philox-4x64-10 blocks for explicit counters (n_blocks x 4 words in, out). */
int mh_debug_philox(mh_ctx* ctx, uint64_t seed, uint64_t stream, int64_t n_blocks,
                    const uint64_t* ctr, uint64_t* out);

/* Stoner-Wohlfarth fall for reduced fields (hx along the axis, hy >= 0 across it) and
 * start angles theta0 in [-pi, pi]: writes n x 6 doubles (theta_c, e_c, theta_o, e_o, e3, two),
 * energies in units of K V (Eq. 2 divided by K V), angles in (-pi, pi]. */
int mh_debug_sw(mh_ctx* ctx, int64_t n, const double* hx, const double* hy,
                const double* theta0, double* out);

/* As mh_debug_sw with the extremum search of step iv chosen: MH_EXTREMA_EXACT (the same
 * as mh_debug_sw) or MH_EXTREMA_SCAN200 (Sec. II.1 step iv taken literally; with fewer
 * than four points found, theta_o = theta_c, e_o = e_c, e3 = NaN, two = 0). MH_EINVAL
 * for another mode or the input errors of mh_debug_sw. */
int mh_debug_sw_mode(mh_ctx* ctx, int32_t extrema_mode, int64_t n, const double* hx,
                     const double* hy, const double* theta0, double* out);

/* Dipolar field of Eq. 1 (T) for moments m (n x 3) of an assembly, as summed by the
 * precision the assembly was created with. B_out: n x 3. */
int mh_debug_field(mh_asm* a, const double* m, double* B_out);

/* ---------------------------------------------------------------------------
 * Continuous-batching server. A scheduler thread admits queued requests in arrival
 * order while their device memory (state, and W for the matrix form) fits the budget,
 * and advances every admitted request together, chunk by chunk, so requests that
 * arrive while others run start as soon as memory frees up and share the launches.
 * Each request runs rounds of up to 64 replicas (256 for the matrix form; replica r
 * uses Philox stream r) until
 * 2 SE <= max(target_rel_err |A|, abs_err_floor) with at least min_replicas, or
 * max_replicas. A request's result is the same alone and in any mix.
 * ------------------------------------------------------------------------- */
typedef struct mh_server mh_server;

typedef struct {
  int64_t n;              /* particles */
  const double* pos;      /* n x 3, m (copied at submit) */
  const double* axes;     /* n_axes_sets x n x 3 (copied at submit) */
  int64_t n_axes_sets;
  mh_params params;
  uint64_t seed;
  double target_rel_err;  /* relative target for 2 SE of the area (e.g. 0.01) */
  double abs_err_floor;   /* absolute floor for 2 SE of the area, J/m^3 (>= 0; 0: none):
                             a request stops once 2 SE <= max(target_rel_err |A|, floor) */
  int64_t min_replicas, max_replicas;
} mh_request;

typedef struct {
  double sar_Wkg, sar_se;   /* W/kg */
  double area_Jm3, area_se; /* J/m^3 */
  int64_t loops;            /* kept loops = replicas x kept periods */
  int64_t replicas;
  uint64_t submit_ns, start_ns, done_ns; /* steady-clock stamps: submit, admission, result */
  int32_t status;           /* MH_OK or an error code */
} mh_result;

/* hbm_budget_bytes: device memory the server may hold for admitted requests. The
 * server runs on a private context of ctx's device. */
int mh_server_create(mh_ctx* ctx, size_t hbm_budget_bytes, mh_server** out);
/* Copies the request; MH_EBUDGET if it can never fit the budget, MH_EOVERLAP/MH_EINVAL
 * for invalid inputs. Thread-safe. */
int mh_server_submit(mh_server* s, const mh_request* req, uint64_t* req_id);
/* Fills *out with the result once the request finished (MH_OK). Before that returns
 * MH_ENOTREADY and fills *out with its progress only: replicas = replicas of the rounds
 * finished so far, submit_ns and start_ns (0 while queued), status MH_ENOTREADY, the
 * rest zero. Thread-safe. */
int mh_server_poll(mh_server* s, uint64_t req_id, mh_result* out);
/* Stops after the admitted requests finish (queued ones are dropped) and frees all. */
int mh_server_destroy(mh_server* s);

/* Launch-shape autotuner. For each particle count in sizes and replica count in
 * replicas, times the candidate shapes of the tiled field kernel (64 or 16 targets per
 * block; source split for 2, 3, 4 or 6 blocks per CU) over full 200-step runs of a
 * synthetic non-overlapping assembly (cubic lattice of spacing 1.25 d, jittered) on
 * the context's device, and stores the fastest in the context's shape table under the
 * buckets of (precision, particle count: powers of two from 256, replica groups:
 * powers of four). Later runs and servers created on the context take their shapes
 * from the table, else from the built-in rule; results stay bitwise the same alone and
 * in any batch for a given table. precision: MH_FP64 or MH_FP32_FIELD (the matrix form
 * has one tile). n_sizes == 0 clears the table. json_path (or NULL) receives the table
 * as JSON. Synchronous; MH_EINVAL for sizes outside [2, 200000], replicas outside
 * [1, 4096], more than 64 of either, or an unwritable path. */
int mh_ctx_autotune(mh_ctx* ctx, int32_t precision, const int64_t* sizes, int32_t n_sizes,
                    const int64_t* replicas, int32_t n_replicas, const char* json_path);

/* Replace the context's shape table by one written by mh_ctx_autotune. MH_EINVAL (table
 * unchanged) when the file is missing, empty or not in that format. */
int mh_ctx_load_shapes(mh_ctx* ctx, const char* json_path);

/* Launch timing (diagnostics for roofline reports). When on, every step-kernel launch
 * is bracketed by a pair of HIP events on the stream it runs on. mh_ctx_get_timing
 * waits for the recorded launches of one kind (0: tiled dipolar-field kernel, 1: resident
 * whole-run launch, 2: interaction-matrix product, 3: per-particle update kernel,
 * 4: update kernel of the interaction-matrix form, 5: mean-magnetisation loop launch),
 * returns their summed duration (ms) and count. mh_ctx_set_timing clears the record. */
int mh_ctx_set_timing(mh_ctx* ctx, int on);
int mh_ctx_get_timing(mh_ctx* ctx, int32_t kind, double* total_ms, int64_t* launches);

/* Kernel durations for roofline reports, on the plan of the assemblies' last run (run
 * together by mh_run_batch or one by mh_run_loops, same replicas; not server requests):
 * the launches of one step of one kernel kind are captured `launches` times (local
 * steps from the first kept step where the run has enough of them), replayed once to
 * warm up and then `reps` times back to back between two HIP events on the context's
 * stream. *us_per_step = mean time of one step's launches of that kind, gaps between
 * back-to-back launches included. kind: 0 tiled dipolar-sum launches, 2 interaction-matrix
 * product, 3 per-particle update of the tiled form, 4 update of the matrix form (the
 * numbering of mh_ctx_get_timing). Kinds 0 and 2 write only the field scratch; kinds 3
 * and 4 advance moments and accumulators, so the assemblies' results are undefined until
 * their next run. Synchronous. MH_EINVAL for an assembly that has not run, a server
 * request, a repeated assembly, launches outside [1, 1000] or reps outside [1, 100000]. */
int mh_time_kernels(mh_asm* const* asms, int32_t count, int32_t kind, int32_t launches,
                    int32_t reps, double* us_per_step);

/* Latency floor of a resident step (diagnostics for the latency-bound small-system
 * form). The step scheme of Sec. II.1 makes every step depend on the previous one (the
 * field of step k uses the moments after step k - 1), so a system run by one workgroup
 * pays at least one exchange through LDS and one barrier per step. This launches one
 * workgroup of the resident kernel's size that runs `steps` such empty steps (each
 * thread reads a neighbour's value of the previous step from one LDS buffer, writes its
 * own to the other, then the barrier) between two HIP events on the context's stream;
 * *us_per_step = their time / steps. Synchronous. MH_EINVAL for steps outside
 * [1, 1e7] or a null argument. */
int mh_time_empty_steps(mh_ctx* ctx, int64_t steps, double* us_per_step);

const char* mh_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* MHKMC_H */
