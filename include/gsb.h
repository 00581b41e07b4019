/*
 * gsb.h -- C ABI of libgsb: simulated bifurcation (bSB, dSB) and its generalisation
 * with individual bifurcation-parameter control (GbSB), for the Ising problem, on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Goto, Hidaka, Tatsumura, "Edge-of-chaos enhanced quantum-inspired algorithm
 * for combinatorial optimization", arXiv 2508.17655.
 *   problem      : minimise E = -1/2 sum_ij J_ij s_i s_j, eq. (1), J symmetric, J_ii = 0.
 *   dynamics     : symplectic-Euler steps, eqs. (3)-(4), perfectly inelastic walls at
 *                  |x| = 1, eq. (5); bifurcation parameter p from 1 to 0 by eq. (6), or
 *                  per-variable by eq. (7) with control strength A (GbSB).
 *   dSB          : J_ij x_j replaced by J_ij sgn(x_j) in eq. (3) (Sec. VI).
 *   parameters   : c = 1/lambda_max(J), x_i(0) ~ U(-0.1, 0.1), y_i(0) = 0 (App. A).
 *
 * Conventions for every entry point:
 *   - Return value is a gsb_status; GSB_OK (0) on success.  On failure a message is
 *     available from gsb_last_error() (thread-local, valid until the next call on the
 *     same thread).  No C++ exception crosses this boundary.
 *   - Pointers documented as "host" point to caller-owned host memory; the library
 *     copies what it needs and keeps no reference after the call returns.  Pointers
 *     documented as "device" point to memory on the current HIP device.
 *   - A context is used by one host thread at a time.  All device work of a context
 *     is enqueued on its stream (gsb_set_stream; default: the null stream).  Calls
 *     that return results to host memory synchronise that stream first.
 *   - After any error a context can still be destroyed.
 */
#ifndef GSB_H
#define GSB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsb_ctx gsb_ctx; /* opaque; owns host copies and device buffers */

typedef enum {
  GSB_OK = 0,
  GSB_EINVAL = -1,        /* argument out of range / null pointer */
  GSB_ENOTSYM = -2,       /* J not exactly symmetric (eq. (1) requires J_ij = J_ji) */
  GSB_EDIAG = -3,         /* nonzero diagonal (eq. (1) requires J_ii = 0) */
  GSB_ENONFINITE = -4,    /* NaN or infinity in J, h or a state array */
  GSB_ENOMEM = -5,        /* device or host allocation failed / workspace too small */
  GSB_EDEVICE = -6,       /* HIP runtime error or a device-side timeout */
  GSB_ESTATE = -7,        /* call out of order (e.g. gsb_energy before gsb_init) */
  GSB_EUNSUPPORTED = -8   /* valid request this build does not provide */
} gsb_status;

/* Variants.  bSB: eqs. (3)-(6).  dSB: bSB with the sign product (Sec. VI).  GbSB: bSB
 * with eq. (7) (the paper's generalised SB).  GdSB: eq. (7) applied to the dSB sign
 * product (the extension the paper's outlook, Sec. VII, asks about). */
typedef enum { GSB_BSB = 0, GSB_DSB = 1, GSB_GBSB = 2, GSB_GDSB = 3 } gsb_variant;

/* Schedules.  LINEAR: p_i(t_0) = 1 and eq. (7) (eq. (6) when A = 0), which reaches 0 at
 * t_M.  CONSTANT: p_i = 1 throughout (used for the stability analysis of App. A). */
typedef enum { GSB_SCHED_LINEAR = 0, GSB_SCHED_CONSTANT = 1 } gsb_schedule;

/* Arithmetic of the coupling product sum_j J_ij q_j (eq. (3)).  The update of p, y, x and
 * the wall is always binary32 (Fig. 2(a) caption).
 *   FP32   : J and q in binary32 on MFMA, binary32 accumulation.
 *   BF16X2 : J in bfloat16; continuous q split into hi = bf16(x), lo = bf16(x - hi);
 *            two MFMA passes, binary32 accumulation.
 *   FP8    : J and q in OCP E4M3 on MFMA, binary32 accumulation.  Requires J_ij in
 *            {0, +1, -1}.  Sign operands (dSB, GdSB) are exact, so the product is exact;
 *            continuous operands (bSB, GbSB) are rounded to E4M3 (nearest even), and the
 *            product of the rounded values is exact.
 *   FIX16  : 16-bit fixed point, the FPGA's JX precision (App. C): q = rint(x 2^14) / 2^14
 *            (round half to even), J in int8; two int8 MFMA passes (q = 256 hi + lo) with
 *            exact int32 accumulation, the sum rounded to binary32 once.  Requires J_ij in
 *            {0, +1, -1}.  An exact continuous product with 14 fraction bits. */
typedef enum { GSB_PREC_FP32 = 0, GSB_PREC_BF16X2 = 1, GSB_PREC_FP8 = 2, GSB_PREC_FIX16 = 3 } gsb_precision;

/* Initial conditions (drawn on the device from the run seed with counter-based
 * SplitMix64, one counter per (replica, stream, spin); replica r's start does not
 * depend on the replica count).
 *   X    : x ~ U(-0.1, 0.1), y = 0 (App. A; default).
 *   XY   : x and y ~ U(-0.1, 0.1).
 *   PM01 : x = +-0.1 with a random sign, y = 0 (the chaos start of Sec. IV).
 *   PAIRS: the trajectory pairs of Sec. IV: replica 2k starts at x = +-0.1 (replica k's
 *          PM01 start), replica 2k+1 at the same x +- 2e-6 (independent random signs,
 *          binary64 sum rounded to binary32 once), y = 0 for both; delta(0) = 1e-6. */
typedef enum { GSB_INIT_X = 0, GSB_INIT_XY = 1, GSB_INIT_PM01 = 2, GSB_INIT_PAIRS = 3 } gsb_init_mode;

/* Options for gsb_set / gsb_get. */
typedef enum {
  GSB_OPT_C = 0,          /* coupling constant c (default 1/lambda_max, App. A) */
  GSB_OPT_PRECISION = 1,  /* gsb_precision (default GSB_PREC_FP8 when J is in {0,+-1},
                             else GSB_PREC_BF16X2) */
  GSB_OPT_INIT_MODE = 2,  /* gsb_init_mode (default GSB_INIT_X) */
  GSB_OPT_LAMBDA_MAX = 3, /* read-only: largest eigenvalue of J (binary64) */
  GSB_OPT_LAMBDA_MIN = 4, /* read-only: smallest eigenvalue of J (binary64) */
  GSB_OPT_N = 5,          /* read-only: number of spins n */
  GSB_OPT_STEP = 6,       /* read-only: current step index m of the run */
  GSB_OPT_REPLICAS = 7,   /* read-only: replicas of the current run */
  GSB_OPT_DT_STABLE = 8,  /* read-only: eq. (13) time step with D_t = 1.25 */
  GSB_OPT_N_DYN = 9,      /* read-only: spins carried by the dynamics (n, plus 1 with a
                             field ancilla); the length of one replica in gsb_state */
  GSB_OPT_STEP_KERNEL = 10 /* step kernel of the FP8 product at n_p <= 2048 (both keep J
                             resident on chip, 256 spins x 32 replicas per workgroup, and
                             compute the same bits): 0 = automatic (default), 1 = one wave
                             per SIMD computes product and update (J in registers),
                             2 = two waves per SIMD, one computing the product (J in
                             registers and LDS), the other the update.  Other precisions
                             and sizes ignore it.  Takes effect at the next gsb_init. */,
  GSB_OPT_GRID_PAD = 11   /* 1 (default): pad the grid of each time-stepping launch to a
                             whole number of rounds of 8 replica groups when that still
                             fits on the device (the padding workgroups exit at once), so
                             that the workgroups of a group are dispatched to one XCD and
                             exchange the operand through its L2; 0: no padding, a group's
                             workgroups may sit on several XCDs and every step then goes
                             through a group counter with device-scope fences (slower; the
                             results are the same bits).  Takes effect at the next launch. */,
  GSB_OPT_LLE_FROM = 12   /* first step m_w whose tangent growth gsb_lle counts (default 0):
                             the estimate becomes ln(|v(t_M)| / |v(t_w)|) / ((M - m_w) dt),
                             with the tangent renormalised to unit norm at t_w, so that the
                             window after the bifurcation (Sec. IV) can be measured apart
                             from the pump's growth through it.  Integer >= 0; gsb_lle
                             rejects a value >= its `steps`. */
} gsb_option;

/* Create a context for the instance (J, h).
 *   J : host, n*n binary32, row-major.  Must be finite, exactly symmetric, zero diagonal
 *       (eq. (1)).  Copied.
 *   h : host, n binary32, or NULL (no field).  A nonzero field adds an ancilla spin
 *       (index n) coupled to spin i by h_i and read as +1 (the whole configuration is
 *       flipped otherwise), so the dynamics stays field-free and the reported energy is
 *       -1/2 s^T J s - h^T s.
 *   n : 1 <= n <= 16384.
 * lambda_max and lambda_min of J are computed in binary64 on the host (Lanczos) when
 * first needed: at gsb_init if c was not set, which then sets c = 1/lambda_max
 * (App. A), or when read with gsb_get.  Needs no device memory yet.
 * Errors: EINVAL, ENONFINITE, ENOTSYM, EDIAG, ENOMEM. */
gsb_status gsb_create(const float* J, const float* h, int32_t n, gsb_ctx** out);

/* Release all host and device resources (device memory bound with gsb_bind_workspace
 * stays owned by the caller).  NULL is ignored. */
void gsb_destroy(gsb_ctx* ctx);

/* Set / read an option (gsb_option).  Errors: EINVAL (unknown option, read-only option,
 * value out of range), EUNSUPPORTED (FP8 precision on J with entries outside {0,+-1}). */
gsb_status gsb_set(gsb_ctx* ctx, int32_t option, double value);
gsb_status gsb_get(gsb_ctx* ctx, int32_t option, double* value);

/* Bind the HIP stream (hipStream_t) all device work of this context is enqueued on.
 * NULL selects the null stream. */
gsb_status gsb_set_stream(gsb_ctx* ctx, void* stream);

/* Device memory a run of `replicas` replicas and `steps` time steps needs at the current
 * precision, in bytes. */
gsb_status gsb_workspace_size(gsb_ctx* ctx, int32_t replicas, int32_t steps, size_t* bytes);

/* Bind caller-owned device memory (e.g. a framework allocation) as the workspace.
 *   device_ptr : device, 256-byte aligned, `bytes` long; must outlive its use by the
 *                context.  NULL unbinds (the library then allocates on demand).
 * A bound workspace smaller than a later run needs makes that run fail with ENOMEM. */
gsb_status gsb_bind_workspace(gsb_ctx* ctx, void* device_ptr, size_t bytes);

/* Start a run: draw the initial state of `replicas` replicas from `seed` and set m = 0
 * of an M = `steps` step schedule.  No time step is taken.
 *   control_strength : A of eq. (7), 0 <= A; ignored (taken as 0) for bSB and dSB.
 *   dt               : time step Delta_t > 0 (App. A: 1.25 for dense random J).
 * Asynchronous on the context's stream.
 * Errors: EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE. */
gsb_status gsb_init(gsb_ctx* ctx, int32_t variant, int32_t schedule, double control_strength,
                    double dt, int32_t replicas, int32_t steps, uint64_t seed);

/* Advance the current run by `count` time steps (m -> m + count, m + count <= M).
 * Asynchronous on the context's stream.  Errors: ESTATE, EINVAL, EDEVICE. */
gsb_status gsb_step(gsb_ctx* ctx, int32_t count);

/* gsb_init followed by all M steps and the final energies (Sec. III evaluates the cut
 * only at the final time).  Asynchronous on the context's stream. */
gsb_status gsb_run(gsb_ctx* ctx, int32_t variant, int32_t schedule, double control_strength,
                   double dt, int32_t replicas, int32_t steps, uint64_t seed);

/* gsb_run without device allocation, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation).  It
 * computes the same bits as gsb_run followed by gsb_energy for the same context and
 * arguments, but every device buffer of the run (the copies of J, the state, the operand
 * buffers, the barrier words, the energy sums and the schedule table) lives in one array
 * of 64 MiB per device that the library holds from its load onto a device until the
 * process ends; no hipMalloc or hipFree is called.  The context's own workspace (bound or
 * allocated) is neither used nor changed.
 *   x        : device, replicas * n_dyn binary32, replica-major (n_dyn = GSB_OPT_N_DYN):
 *              x at t_M.
 *   energies : device, replicas doubles: the eq. (1) energies of sgn(x) at t_M.
 *   other arguments as gsb_run.
 * Limit: the run must fit in the array (what gsb_workspace_size reports for the same
 * replicas and steps, at most 64 MiB; for example n = 2000 with 1024 replicas in the FP8
 * precision); a larger run fails with EINVAL before any device work.
 * All calls on one device share that device's array, which keeps the last call's contents
 * (a later call by the same context reuses its J there, any other call overwrites it):
 * calls that overlap in time on one device race and give undefined results, so serialise
 * them (one host thread, one stream at a time).  Enqueued on the context's stream; then
 * synchronises it and checks the barrier status.  Afterwards the context has no current run
 * (ESTATE for gsb_step, gsb_energy, gsb_state, ...).
 * Errors: EINVAL, EUNSUPPORTED, EDEVICE. */
gsb_status gsb_run_noalloc(gsb_ctx* ctx, int32_t variant, int32_t schedule, double control_strength, double dt,
                           int32_t replicas, int32_t steps, uint64_t seed, float* x, double* energies);

/* Ising energies, eq. (1), of s = sgn(x) (sgn(0) = +1) at the current step, one per
 * replica.  energies: host, `replicas` doubles.  Exact for integer J; binary64
 * accumulation otherwise.  Synchronises the stream.  Errors: ESTATE, EINVAL, EDEVICE. */
gsb_status gsb_energy(gsb_ctx* ctx, double* energies);

/* The replica with the lowest energy (ties to the lowest index) and its spins.
 *   spins   : host, n int8 values in {-1, +1}, or NULL.
 *   energy  : host, or NULL.   replica : host, or NULL.
 * Synchronises the stream.  Errors: ESTATE, EDEVICE. */
gsb_status gsb_best(gsb_ctx* ctx, int8_t* spins, double* energy, int32_t* replica);

/* All spins s = sgn(x) at the current step.  spins: host, replicas*n int8 (replica-major).
 * Synchronises the stream. */
gsb_status gsb_spins(gsb_ctx* ctx, int8_t* spins);

/* Copy out the state at the current step.  x, y, p: host, replicas*n_dyn binary32 each
 * (replica-major; n_dyn = GSB_OPT_N_DYN), any of them NULL to skip; m: host or NULL.
 * Synchronises. */
gsb_status gsb_state(gsb_ctx* ctx, float* x, float* y, float* p, int32_t* m);

/* Replace the state of the current run (checkpoint resume): x, y, p host arrays as in
 * gsb_state, all non-NULL and finite, |x| <= 1; 0 <= m <= M.  Synchronises.
 * Errors: ESTATE, EINVAL, ENONFINITE, EDEVICE. */
gsb_status gsb_set_state(gsb_ctx* ctx, const float* x, const float* y, const float* p, int32_t m);

/* gsb_state and gsb_set_state with the arrays in device memory (e.g. a framework's tensors
 * on the context's device), so that a checkpointed trajectory (the differentiation path)
 * keeps its state on the device.  Layout as for the host versions: replicas * n_dyn
 * binary32 each, replica-major, caller-owned.  The copies run on the context's stream
 * (gsb_set_stream); order the caller's own work on the arrays with it.  gsb_state_device
 * synchronises and checks the barrier status like gsb_state.  gsb_set_state_device makes
 * gsb_set_state's checks in a kernel (non-finite entries: ENONFINITE; |x| > 1: EINVAL,
 * the state left as it was) and synchronises.
 * Errors: ESTATE, EINVAL, ENONFINITE, EDEVICE. */
gsb_status gsb_state_device(gsb_ctx* ctx, float* x, float* y, float* p, int32_t* m);
gsb_status gsb_set_state_device(gsb_ctx* ctx, const float* x, const float* y, const float* p, int32_t m);

/* Normalised distance of the trajectory pairs, eq. (8) (Sec. IV), at the current step:
 * delta_k = sqrt(sum_i (x_i(2k) - x_i(2k+1))^2 / (4 n)) over the n spins of the instance
 * (a field ancilla excluded), for k < replicas/2.  Meaningful for runs started with
 * GSB_INIT_PAIRS.  out: host, replicas/2 doubles (binary64).  Synchronises.
 * Errors: ESTATE (no run), EINVAL (NULL, fewer than 2 replicas), EDEVICE. */
gsb_status gsb_delta(gsb_ctx* ctx, double* out);

/* Largest-Lyapunov-exponent estimates (a chaos measure beside eq. (8); not in the paper).
 * Runs `replicas` replicas of bSB or GbSB (continuous product; the sign product's
 * derivative is 0) for M = `steps` steps in the binary32 (FP32) form, each with the
 * forward derivative of every step (of eqs. (7), (3), (4), (5): dp' = dp (1 - f r_m) +
 * 2 A x dx p r_m with f = 1 - A x^2; dy' = dy - (dp' x + p' dx) dt + c dt (J dx);
 * dx' = dx + dy' dt; dx' = dy' = 0 where the wall acts).  The J dx products share the
 * GEMM of the J x products (2 replicas' worth of columns per replica).
 *   variant          : GSB_BSB or GSB_GBSB.     schedule, dt, seed: as gsb_init; the
 *                      primal start of replica r equals gsb_init's for the same seed and
 *                      GSB_OPT_INIT_MODE.
 *   control_strength : A for every replica when A_per_replica is NULL.
 *   A_per_replica    : host, `replicas` doubles >= 0, or NULL (a sweep over A in one run).
 *   tangent_seed     : starting tangent dx_i = +-1 (bit 63 of SplitMix64 output
 *                      r*n_dyn + i + 1 of tangent_seed), dy = dp = 0, scaled to unit norm
 *                      over (dx, dy, dp).
 *   renorm_every     : steps between rescalings of the tangent to unit norm (>= 1); the
 *                      logarithms of the norms are summed in binary64.
 *   lle              : host, `replicas` doubles: ln(|v(t_M)| / |v(t_w)|) / ((M - m_w) dt)
 *                      with m_w = GSB_OPT_LLE_FROM (0 by default), or -inf when every
 *                      component of the tangent reached a wall.
 *   state_out        : host, 6 * replicas * n_dyn floats or NULL: x, y, p, dx, dy, dp at
 *                      t_M (the tangent at unit norm), each replica-major.
 * Uses the context's workspace; afterwards the context has no current run (ESTATE for
 * gsb_step, gsb_energy, ...).  gsb_last_step_ms reports its device time.  Synchronises.
 * Errors: EINVAL, ENOMEM, EUNSUPPORTED, EDEVICE. */
/* Device memory gsb_lle needs for `replicas` replicas and `steps` steps, in bytes. */
gsb_status gsb_lle_workspace_size(gsb_ctx* ctx, int32_t replicas, int32_t steps, size_t* bytes);

gsb_status gsb_lle(gsb_ctx* ctx, int32_t variant, int32_t schedule, double control_strength,
                   const double* A_per_replica, double dt, int32_t replicas, int32_t steps, uint64_t seed,
                   uint64_t tangent_seed, int32_t renorm_every, double* lle, float* state_out);

/* Reverse derivative (vector-Jacobian product) of the next `count` steps of the current
 * run, without advancing it: given the cotangents of x, y, p after those steps, return
 * the cotangents of x, y, p at the current step.  bSB/GbSB runs in the FP32 precision
 * only (the sign product and the E4M3 rounding are piecewise constant).  The reverse
 * step is the transpose of the forward derivative documented at gsb_lle; J symmetric,
 * so it uses the same product.  The library recomputes the `count` steps from the
 * current state and keeps every step's input state on the device (12 bytes per element
 * and step, allocated and kept by the context until gsb_destroy): checkpoint long
 * trajectories in segments (restore each segment's start with gsb_set_state).
 *   xb, yb, pb : host, replicas * n_dyn binary32 each, replica-major; overwritten.
 * Synchronises.  Errors: ESTATE, EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE. */
gsb_status gsb_vjp(gsb_ctx* ctx, int32_t count, float* xb, float* yb, float* pb);

/* gsb_vjp with the cotangents in device memory (replicas * n_dyn binary32 each, replica-
 * major, caller-owned, overwritten), copied on the context's stream.  Synchronises.
 * Errors: as gsb_vjp. */
gsb_status gsb_vjp_device(gsb_ctx* ctx, int32_t count, float* xb, float* yb, float* pb);

/* Device time of the last gsb_step/gsb_run time stepping (the persistent step kernel
 * launches), in milliseconds, measured with HIP events on the context's stream.
 * Synchronises the stream. */
gsb_status gsb_last_step_ms(gsb_ctx* ctx, double* ms);

/* ---- Batched instances ---------------------------------------------------------------
 * A batch holds `count` Ising instances of (possibly) different sizes n_k, each with J in
 * {0, +1, -1} and no field, and runs `replicas` replicas of every instance in ONE
 * persistent kernel launch.  This is batch processing (Sec. VI: several problems solved
 * side by side) generalised to instances of different sizes.  Every instance computes
 * exactly what a context in GSB_PREC_FP8 computes for it (the E4M3 product of eq. (3),
 * or the sign product of dSB/GdSB, with the binary32 update of eqs. (3)-(7)): bit for
 * bit the same x, y, p and energies for the same J, variant, A, c, dt, steps and seed
 * seed + k (k = the instance index), with GSB_OPT_INIT_MODE = the batch's init mode.
 *
 * Placement: each replica group of an instance (a tile of 64, 128 or 256 spin rows by
 * 8192 / rows replicas; see GSB_BATCH_TILE_ROWS) is a gang of n_p / rows workgroups
 * that run together; gangs wait in one queue per XCD, balanced by the host (longest
 * processing time first), and a workgroup that finishes a gang takes the next slot of
 * its queue.  gsb_batch_autotune measures the step time of every instance at each tile
 * shape on the device and later runs use the fastest one.
 *
 * Same conventions as the rest of this header; a batch is used by one host thread at a
 * time, except gsb_batch_set_coupling, which may run on several threads at once for
 * different instances (the eigenvalue estimates then run in parallel). */
typedef struct gsb_batch gsb_batch; /* opaque; owns host tables and device buffers */

typedef enum {
  GSB_BATCH_C = 0,          /* per instance: c (default 1/lambda_max, App. A) */
  GSB_BATCH_DT = 1,         /* per instance: dt (default eq. (13) with D_t = 1.25) */
  GSB_BATCH_LAMBDA_MAX = 2, /* per instance, read-only: lambda_max (when it was computed) */
  GSB_BATCH_LAMBDA_MIN = 3, /* per instance, read-only: lambda_min (when it was computed) */
  GSB_BATCH_TILE_ROWS = 4,  /* per instance: 64, 128 or 256 spin rows per workgroup tile;
                               0 (default) = automatic: the fastest measured tile, else the
                               smallest whose gang fits in one XCD's workgroups */
  GSB_BATCH_STEP_US = 5,    /* per instance, read-only: measured microseconds per step of one
                               replica group at the current tile (0 = not measured) */
  GSB_BATCH_N = 6,          /* per instance, read-only: n */
  GSB_BATCH_GRAPH = 7,      /* batch-wide (k = -1): 1 = gsb_batch_run captures its launch
                               sequence in a HIP graph once and replays it while the run's
                               arguments and the batch are unchanged (default 0) */
  GSB_BATCH_INIT_MODE = 8,  /* batch-wide (k = -1): gsb_init_mode (default GSB_INIT_X) */
  GSB_BATCH_COUNT = 9,      /* batch-wide, read-only: count */
  GSB_BATCH_REPLICAS = 10,  /* batch-wide, read-only: replicas */
  GSB_BATCH_GRID = 11,      /* batch-wide, read-only: workgroups of the persistent launch */
  GSB_BATCH_OCCUPANCY = 12  /* batch-wide: workgroups per CU of the launch, 1 or 2 (with 2, one
                               workgroup's update and barrier overlap the other's product,
                               with half the LDS and a shallower prefetch each); 0 (default) =
                               chosen by gsb_batch_autotune, 1 until it runs */
} gsb_batch_option;

/* Create a batch of `count` instances (1 <= count <= 65536) of sizes n[k]
 * (1 <= n[k] <= 8192; host array, copied), `replicas` replicas each (1..65536).
 * Needs no device memory yet.  Errors: EINVAL, ENOMEM. */
gsb_status gsb_batch_create(int32_t count, const int32_t* n, int32_t replicas, gsb_batch** out);

/* Release the batch (a bound workspace stays the caller's).  NULL is ignored. */
void gsb_batch_destroy(gsb_batch* batch);

/* Bind the HIP stream all device work of the batch is enqueued on (NULL: null stream). */
gsb_status gsb_batch_set_stream(gsb_batch* batch, void* stream);

/* Device memory the batch needs (all instances' J, states, operands, energies), bytes. */
gsb_status gsb_batch_workspace_size(gsb_batch* batch, size_t* bytes);

/* Bind caller-owned device memory (256-byte aligned, at least gsb_batch_workspace_size
 * bytes) before the first gsb_batch_set_coupling; otherwise the library allocates it
 * there.  Errors: EINVAL, ENOMEM (too small), ESTATE (couplings already set). */
gsb_status gsb_batch_bind_workspace(gsb_batch* batch, void* device_ptr, size_t bytes);

/* Give instance k its coupling matrix and parameters.
 *   J  : host, n_k * n_k binary32, row-major, entries in {0, +1, -1}, exactly symmetric,
 *        zero diagonal (eq. (1)).  Uploaded (as FP4 in the fragment layout of the FP8
 *        product) before the call returns.
 *   c  : > 0, or <= 0 for c = 1/lambda_max (App. A).
 *   dt : > 0, or <= 0 for eq. (13), dt = 1.25 sqrt(2 / (1 - lambda_min / lambda_max)).
 * lambda_max and lambda_min are estimated on the host (Lanczos, binary64) only when c or
 * dt is left to the library.  Synchronises the stream.
 * Errors: EINVAL, EDIAG, ENOTSYM, ENONFINITE, EUNSUPPORTED (entries outside {0, +-1}),
 * ENOMEM, EDEVICE. */
gsb_status gsb_batch_set_coupling(gsb_batch* batch, int32_t k, const float* J, double c, double dt);

/* Set / read an option (gsb_batch_option) of instance k, or of the batch with k = -1.
 * Errors: EINVAL (unknown option, bad value or index), ESTATE (no coupling yet / value
 * not computed), EDEVICE. */
gsb_status gsb_batch_set(gsb_batch* batch, int32_t k, int32_t option, double value);
gsb_status gsb_batch_get(gsb_batch* batch, int32_t k, int32_t option, double* value);

/* Measure, on the device, the step time of every instance at each tile shape (64, 128
 * and 256 rows; shapes whose gang does not fit in one XCD are skipped) and each
 * occupancy (1 and 2 workgroups per CU) with trial runs of `trial_steps` steps of the
 * whole batch, keep the results for later runs (tile choice and queue balance), and
 * choose the occupancy whose whole-batch trial with its fastest tiles is quicker.
 * Instances with a fixed GSB_BATCH_TILE_ROWS keep it, a fixed GSB_BATCH_OCCUPANCY too.
 * Leaves no current run.  Synchronises.  Errors: EINVAL, ESTATE, EUNSUPPORTED, EDEVICE. */
gsb_status gsb_batch_autotune(gsb_batch* batch, int32_t variant, double control_strength, int32_t trial_steps,
                              uint64_t seed);

/* Run every instance: starting states (instance k from seed + k), M = `steps` steps of
 * `variant` with control strength A (ignored for bSB and dSB) in one persistent launch,
 * then the energies and best replica of every instance.  Asynchronous on the stream.
 * Errors: EINVAL, ESTATE (an instance without coupling), EUNSUPPORTED (an instance too
 * large for one XCD's workgroups), ENOMEM, EDEVICE. */
gsb_status gsb_batch_run(gsb_batch* batch, int32_t variant, double control_strength, int32_t steps, uint64_t seed);

/* Energies, eq. (1), of the `replicas` replicas of instance k after the last run
 * (exact; host, `replicas` doubles).  Synchronises.  Errors: EINVAL, ESTATE, EDEVICE. */
gsb_status gsb_batch_energy(gsb_batch* batch, int32_t k, double* energies);

/* Lowest energy and its replica (ties to the lowest index) of every instance after the
 * last run; host arrays of `count` entries, either may be NULL.  Synchronises. */
gsb_status gsb_batch_best(gsb_batch* batch, double* energy, int32_t* replica);

/* State of instance k after the last run: x, y, p host arrays of replicas * n_k binary32
 * (replica-major), any may be NULL.  Synchronises. */
gsb_status gsb_batch_state(gsb_batch* batch, int32_t k, float* x, float* y, float* p);

/* Device time of the last gsb_batch_run in milliseconds (HIP events on the stream): the
 * persistent step kernel alone, or, with GSB_BATCH_GRAPH, the whole graph (starting
 * states, steps, energies).  Synchronises the stream. */
gsb_status gsb_batch_last_ms(gsb_batch* batch, double* ms);

/* The queue plan gsb_batch_run uses, for inspection: `units` units (here: instances),
 * unit u being gangs[u] gangs of width[u] workgroups that take cost[u] each, over
 * `queues` queues of `workers` workgroups.  Longest processing time first: units in
 * decreasing order of gangs * width * cost, each to the queue with the least work so
 * far; queue[u] receives the queue and rank[u] the position within it (decreasing cost,
 * then width, then index).  Host only.  Errors: EINVAL, EUNSUPPORTED (width > workers). */
gsb_status gsb_batch_plan(int32_t units, const int32_t* width, const int32_t* gangs, const double* cost,
                          int32_t queues, int32_t workers, int32_t* queue, int32_t* rank);

/* Encode `count` binary32 values as the operand of the coupling product sum_j J_ij x_j
 * of eq. (3) sees them in precision `precision`, with the encoders the step kernels
 * use for their operand stores.  discrete != 0 encodes the sign s(x) (+1 for x >= 0,
 * including -0.0) instead, the dSB/GdSB operand (Sec. VI).  Output, value-major:
 *   GSB_PREC_FP8    : count OCP E4M3 bytes (round to nearest, ties to even)
 *   GSB_PREC_BF16X2 : count bfloat16 hi, then count bfloat16 lo, with hi = bf16(x) and
 *                     lo = bf16(x - hi), both rounded to nearest even
 *   GSB_PREC_FIX16  : count int8 hi, then count int8 lo, with rint(x 2^14) = 256 hi + lo
 *                     (16-bit fixed point, the JX module's precision class, App. C)
 *   GSB_PREC_FP32   : count binary32 values
 * The value the product uses is the decoded sum (hi + lo, or (256 hi + lo) 2^-14).  For
 * |x| <= 1, the range the wall of eq. (5) keeps x in, every form is defined; FIX16 needs
 * |x| <= 1.  x, out: device pointers, 4-byte aligned, not overlapping; out holds count
 * bytes (FP8), 4 count (BF16X2, FP32) or 2 count (FIX16).  Asynchronous on `stream`
 * (hipStream_t, NULL = the null stream); allocates nothing.  count = 0 returns GSB_OK
 * without touching the device.  Errors: EINVAL (precision, count < 0, NULL or misaligned
 * pointers), EDEVICE. */
gsb_status gsb_encode_operand(int32_t precision, int32_t discrete, const float* x, int64_t count, void* out,
                              void* stream);

/* Message of the last failed call on this thread ("" if none). */
const char* gsb_last_error(void);

/* Library version string. */
const char* gsb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GSB_H */
