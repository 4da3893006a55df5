/*
 * fnlb — fluctuating two-species D2Q9 lattice Boltzmann on MI355X (gfx950).
 *
 * C ABI of the GPU library.  The method is the fluctuating multicomponent
 * lattice Boltzmann scheme of Belardinelli, Sbragaglia, Benzi and Ciliberto,
 * "Lattice Boltzmann Simulations of Non-Equilibrium Fluctuations in a
 * Non-Ideal Binary Mixture" (arXiv:1808.05168): a binary mixture between two
 * walls at z = +-L/2 with periodic x (Sec. III.A), an imposed linear
 * concentration profile c_0(z) = 1/2 + z grad_c0 (Fig. 1), the non-ideal
 * interaction force of Eq. (11), the non-equilibrium acceleration of Eq. (12)
 * with the a_* correction of the footnote to Eq. (13), MRT relaxation
 * (Eq. (15), Table I) and thermal noise in the non-conserved moments
 * (Eqs. (22)-(23)).  The observables are the structure factors of the
 * concentration and density fluctuations (Appendix, Eqs. (A1)-(A4)) and the
 * mean pressure (Eq. (24), Sec. IV.C).
 *
 * Conventions shared by every call:
 *  - All functions return FNLB_OK (0) or a negative FNLB_E* code; no call
 *    throws.  Errors are sticky per handle: once a call failed with
 *    FNLB_EDEVICE or FNLB_EWATCHDOG, later calls on that handle return it.
 *  - Device buffers (state, accumulators, workspace) are allocated and owned
 *    by the caller, sized by fnlb_bytes_required(), 256-byte aligned, and must
 *    outlive the handle.  The library allocates no device memory.  It owns
 *    only small host metadata and the streams, events and graphs of its
 *    captured sampling periods, freed by fnlb_destroy().
 *  - Work is enqueued asynchronously on the caller's HIP stream; read_* calls
 *    synchronise that stream and copy into caller-allocated host arrays.
 *  - One handle is used from one host thread at a time.
 */
#ifndef FNLB_H
#define FNLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define FNLB_OK 0
#define FNLB_EINVAL (-1)    /* invalid argument or parameter */
#define FNLB_ENOMEM (-2)    /* a caller buffer is smaller than required */
#define FNLB_EDEVICE (-3)   /* a HIP runtime call failed */
#define FNLB_EWATCHDOG (-4) /* non-finite or non-physical state detected */
#define FNLB_ESTATE (-5)    /* call not valid in the handle's current state */

/* ---- precision of the stored populations ---- */
#define FNLB_FP64 0     /* populations stored and updated in FP64 */
#define FNLB_FP32_DEV 1 /* FP32 storage of deviations from w_l rho_ref^S(z);
                           collision in FP32, observables and accumulators in
                           FP64 */

/* ---- option flags (fnlb_options.flags) ---- */
#define FNLB_ASTAR 1         /* a_* correction of the footnote to Eq. (13) */
#define FNLB_WALL_UZ_FIX 2   /* U_z = 0 on the wall rows every step (Sec. III.A) */
#define FNLB_NOISE_LOC 4     /* noise amplitudes of Eqs. (22)-(23) from local
                                densities instead of the reference values */
#define FNLB_FORCE_LITERAL 8 /* first-order forcing moments rho^S a^S without
                                the (1 - lambda_d/2) factor (diagnostic) */
#define FNLB_NO_GRAPH 16      /* execution only: launch every step directly
                                instead of replaying captured graphs */
#define FNLB_SAMPLE_VELOCITY 32 /* also sample U_x and U_z (fields 2, 3): the
                                barycentric velocity of Eq. (10) after the wall
                                fix, for S_U(q) of Sec. IV.A, Eq. (31) */
#define FNLB_TWO_STEP 64       /* execution only: advance pairs of steps with the
                                two-step kernel (FP32_DEV storage and every
                                Lx <= 512, else FNLB_EINVAL) */
#define FNLB_ONE_STEP 128      /* execution only: one step per launch, also after
                                fnlb_autotune */
#define FNLB_DEFAULT_FLAGS (FNLB_ASTAR | FNLB_WALL_UZ_FIX)

/* ---- fields of the structure factor ---- */
#define FNLB_FIELD_C 0   /* delta c   = rho^A/rho - c_0(z) */
#define FNLB_FIELD_RHO 1 /* delta rho = rho - rho_bar */
#define FNLB_FIELD_UX 2  /* U_x (needs FNLB_SAMPLE_VELOCITY) */
#define FNLB_FIELD_UZ 3  /* U_z (needs FNLB_SAMPLE_VELOCITY) */

/* One lattice ("replica").  Sec. III.A: Lx x Lz nodes, x periodic, walls half
 * a link outside rows 0 and Lz-1, reference density rho_bar, c_bar0 = 1/2. */
typedef struct {
  int32_t Lx, Lz;   /* Lx >= 2 columns (periodic), Lz >= 2 fluid rows */
  double rho0;      /* reference total density rho_bar > 0 */
  double grad_c0;   /* imposed concentration gradient; |grad_c0| * Lz < 1 */
  double kT;        /* thermal energy >= 0 (0: noiseless) */
  double G;         /* non-ideal coupling of Eq. (11), >= 0 */
  double tau_d;     /* 1/lambda_d: moments a = 1,2 (Eq. (16)); D = (tau_d - 1/2)/3 */
  double tau_s;     /* 1/lambda_s: moments a = 4,5 (Eq. (17)); nu = (tau_s - 1/2)/3 */
  double tau_e;     /* 1/lambda_e: moment a = 3 */
  double tau_q;     /* 1/lambda_Q: moments a = 6,7 */
  double tau_eps;   /* 1/lambda_eps: moment a = 8; every tau > 1/2 */
  uint64_t seed;    /* Philox4x32-10 key of this replica's noise */
} fnlb_replica_params;

typedef struct {
  int32_t precision;    /* FNLB_FP64 or FNLB_FP32_DEV */
  int32_t sample_every; /* > 0: inside fnlb_step, the state f(t) is sampled
                           (structure factors and pressure) before the step
                           t -> t+1 whenever t >= 1 and t % sample_every == 0;
                           0: sampling only through
                           fnlb_accumulate_structure_factor() */
  int32_t flags;        /* FNLB_* option bits; FNLB_DEFAULT_FLAGS recommended */
  int32_t chunk_rows;   /* rows per work item of the step kernel; 0 = automatic
                           (autotuned value if one was stored for this shape) */
} fnlb_options;

typedef struct fnlb_handle fnlb_handle;

/* Bytes of the three caller-owned device buffers for n_rep replicas:
 *   state: two ping-pong copies of 2 species x 9 populations per node, FP64 or
 *          FP32 per options->precision (layout internal; read it through
 *          fnlb_read_populations);
 *   accum: FP64 accumulators (structure factors and pressure sums);
 *   work:  sample fields, FFT staging, twiddles, tables and reduction partials.
 * Returns FNLB_EINVAL for invalid parameters (the checks of fnlb_init). */
int fnlb_bytes_required(const fnlb_replica_params* reps, int32_t n_rep,
                        const fnlb_options* options, size_t* state_bytes,
                        size_t* accum_bytes, size_t* work_bytes);

/* Creates a handle over the caller's buffers, uploads the replica tables,
 * sets time t = 0, initialises every replica to the state of rest on the
 * imposed profile (f^S_l = w_l rho_0^S(z), rho_0^A = rho_bar c_0(z),
 * rho_0^B = rho_bar (1 - c_0(z)), U = 0; Fig. 1) and clears the accumulators.
 * hip_stream is a hipStream_t (NULL = default stream).  Synchronises that
 * stream before returning (the host-side tables it uploads are temporary).
 * Unless FNLB_NO_GRAPH is set, it also captures the HIP graphs of the
 * sampling period that fnlb_step replays (periods up to 1024 steps), so that
 * fnlb_step itself never captures or instantiates a graph.
 * Errors: FNLB_EINVAL (parameters, null or unaligned buffers), FNLB_ENOMEM
 * (a buffer smaller than fnlb_bytes_required), FNLB_EDEVICE. */
int fnlb_init(const fnlb_replica_params* reps, int32_t n_rep,
              const fnlb_options* options, void* d_state, size_t state_bytes,
              void* d_accum, size_t accum_bytes, void* d_work,
              size_t work_bytes, void* hip_stream, fnlb_handle** out);

/* For callers that cannot allocate device memory (code that will run under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * fnlb_init without the caller's workspace.  The workspace is instead a static
 * device array of FNLB_STATIC_WORK_BYTES inside the library, one per GPU,
 * held from the library's load until the process ends; the caller still
 * passes the state and accumulator buffers (fnlb_bytes_required sizes them)
 * and the stream.  The handle launches every step directly on that stream, as
 * with FNLB_NO_GRAPH (which is implied), so a caller may capture fnlb_step into
 * a graph of its own.  Neither this call nor the handle's other calls
 * allocate device memory.  The array is shared by everything on one GPU: only
 * one handle made by this call may exist per device at a time (a second call
 * on that device returns FNLB_ESTATE until fnlb_destroy of the first), and
 * the array keeps the last handle's contents, which this call overwrites
 * before use.  Work of such a handle that overlaps other use of the array on
 * the same GPU races.  The device is the current HIP device.
 * Such a handle keeps the row spectra of fewer samples per column pass than
 * fnlb_init's (the workspace fnlb_bytes_required reports holds 16; here as
 * many as fit, down to one); its results are the same.
 * Errors: as fnlb_init; FNLB_ENOMEM also when even a workspace of one
 * sample's spectra exceeds FNLB_STATIC_WORK_BYTES; FNLB_ESTATE as above. */
#define FNLB_STATIC_WORK_BYTES (128u << 20)
int fnlb_init_static_work(const fnlb_replica_params* reps, int32_t n_rep,
                          const fnlb_options* options, void* d_state,
                          size_t state_bytes, void* d_accum, size_t accum_bytes,
                          void* hip_stream, fnlb_handle** out);

/* Advances every replica by n >= 0 time steps of Eq. (6): per node,
 * densities, non-ideal and non-equilibrium forces, wall U_z fix, barycentric
 * velocity (Eq. (10)), MRT collision with forcing moments and noise (Eq. (14)),
 * then streaming with mid-way bounce-back at the walls and periodic x.
 * Samples according to options->sample_every.  All replicas advance in one
 * kernel launch per step, or per pair of steps with the two-step kernel (which
 * keeps the state of the middle time in LDS; a pair never spans a sample time
 * other than its first, and results equal those of single steps to FP32
 * rounding).  Whole sampling periods (sample_every steps, or 16
 * steps without sampling) that start on a period boundary are replayed from
 * HIP graphs captured by fnlb_init or fnlb_autotune (periods longer than 1024
 * steps: on first use; none with FNLB_NO_GRAPH): one of up to 16 periods while
 * that many remain (within 1024 steps), else one of two periods, else one of a
 * single period.  In a
 * graph the transforms of each sample run on a branch of their own beside the
 * steps that follow it, joined before the next sample.  The row transforms of
 * up to 16 samples are kept and their column transforms done in one pass,
 * adding the samples in time order; every sample of a call is in the
 * accumulators when the call's work completes, and results are identical
 * with or without graphs.  Asynchronous: all of it is ordered on the caller's
 * stream. */
int fnlb_step(fnlb_handle* h, int64_t n);

/* Chooses the step kernel and the number of rows each of its work items
 * covers by timing steps_per_trial >= 1 launches of each candidate, twice in
 * turn: the one-step kernel with 1 to 128 rows and, where it fits (FP32_DEV,
 * every Lx <= 512), the two-step kernel with 8 to 256 rows (FNLB_ONE_STEP or
 * FNLB_TWO_STEP restrict the choice to one kernel).  It keeps the candidate
 * whose faster round takes the least time per step, for this handle and, for
 * the rest of the process, for any handle with the same precision and set of
 * lattice shapes created with options->chunk_rows = 0.  Trial launches read
 * the current state and write the spare copy, so the state and the time are
 * unchanged.  The period graphs are captured again for the choice.
 * Synchronises the stream; *chunk_rows_out (nullable) receives the rows. */
int fnlb_autotune(fnlb_handle* h, int32_t steps_per_trial, int32_t* chunk_rows_out);

/* The autotuner's choices, per precision and multiset of lattice shapes, are
 * kept for the life of the process and may be saved to and loaded from a
 * text file keyed also by the GPU architecture (entries of other
 * architectures in the file are kept by save and ignored by load).
 * fnlb_tune_lookup: *found = 1 and the stored choice if there is one for
 * these replicas and precision, else *found = 0.
 * fnlb_tune_cache_save: writes every choice of this process for the current
 * device's architecture to path (replaced atomically).  FNLB_EINVAL if the
 * file cannot be written.
 * fnlb_tune_cache_load: adds the file's entries for the current device's
 * architecture to the process's choices.  FNLB_EINVAL if the file cannot be
 * read or is not a tuning file. */
int fnlb_tune_lookup(const fnlb_replica_params* reps, int32_t n_rep, int32_t precision,
                     int32_t* found, int32_t* steps_per_launch, int32_t* chunk_rows);
int fnlb_tune_cache_save(const char* path);
int fnlb_tune_cache_load(const char* path);

/* The launch configuration in use: steps each launch of the state advances
 * (1, or 2 with the two-step kernel) and rows per work item.  Either pointer
 * may be NULL. */
int fnlb_launch_config(const fnlb_handle* h, int32_t* steps_per_launch, int32_t* chunk_rows);

/* Samples the current state f(t) of every replica now: adds |Phi(q)|^2,
 * Re Phi(q), Im Phi(q) of delta c and delta rho (and of U_x, U_z with
 * FNLB_SAMPLE_VELOCITY), with
 * Phi(q) = (Lx Lz)^{-1/2} sum_{x,j} delta phi(x,j) exp(-i (q_x x + q_z j)),
 * q_x = 2 pi k_x / Lx, q_z = 2 pi k_z / Lz, to the structure-factor
 * accumulators, and the spatial mean of P - P_ref (its square, and its row
 * means) to the pressure accumulators.  Asynchronous. */
int fnlb_accumulate_structure_factor(fnlb_handle* h);

/* Copies the structure-factor sums of replica rep, field FNLB_FIELD_C,
 * FNLB_FIELD_RHO, or (with FNLB_SAMPLE_VELOCITY, else FNLB_EINVAL)
 * FNLB_FIELD_UX / FNLB_FIELD_UZ, into host arrays of Lz * (Lx/2 + 1) doubles laid out
 * [k_z][k_x] (k_x = 0..Lx/2); any of the three may be NULL.  S(q) =
 * sum_abs2/n - (sum_re/n)^2 - (sum_im/n)^2.  Synchronises the stream. */
int fnlb_read_structure_factor(fnlb_handle* h, int32_t rep, int32_t field,
                               double* sum_abs2, double* sum_re,
                               double* sum_im, int64_t* n_samples);

/* Copies the pressure sums of replica rep: sum over samples of the spatial
 * mean of P - P_ref, of its square, and (profile_sum, nullable, Lz doubles) of
 * the row means.  P(r) = rho/3 + (G/4) sum_{l>=1} w_l |c_l|^2 [rho^A(r)
 * rho^B(r+c_l) + rho^B(r) rho^A(r+c_l)] (half trace of the pressure tensor;
 * equals Eq. (24) on a uniform state), P_ref = rho_bar/3 + G rho_bar^2/12.
 * Synchronises the stream. */
int fnlb_read_pressure(fnlb_handle* h, int32_t rep, double* sum_dP,
                       double* sum_dP2, double* profile_sum,
                       int64_t* n_samples);

/* Copies the populations f(t) of replica rep as FP64 full values (not
 * deviations) into a host array laid out [species][l][z][x] (2*9*Lz*Lx).
 * Synchronises the stream. */
int fnlb_read_populations(fnlb_handle* h, int32_t rep, double* out);

/* Overwrites the populations of replica rep from a host array in the layout
 * of fnlb_read_populations (FP32_DEV rounds the deviations to FP32).
 * Synchronises the stream. */
int fnlb_write_populations(fnlb_handle* h, int32_t rep, const double* in);

/* Clears all structure-factor and pressure accumulators and the sample count.
 * Asynchronous. */
int fnlb_reset_accumulators(fnlb_handle* h);

/* Replaces the physical parameters and seeds of every replica (n_rep and each
 * Lx, Lz must equal the handle's, else FNLB_EINVAL) and starts over as
 * fnlb_init does: rest state on the imposed profile, t = 0, accumulators
 * cleared.  Buffers, work items, autotuned row ranges and captured graphs are
 * kept, so a caller that evaluates many parameter sets on one shape (a
 * parameter scan, an optimisation loop) creates one handle.  Synchronises the
 * stream. */
int fnlb_reinit(fnlb_handle* h, const fnlb_replica_params* reps, int32_t n_rep);

/* Current time t (number of steps taken since init). */
int fnlb_get_time(const fnlb_handle* h, int64_t* t);

/* Sets the time counter (keys the noise and the sampling schedule), e.g. to
 * continue a run after fnlb_write_populations.  t >= 0. */
int fnlb_set_time(fnlb_handle* h, int64_t t);

/* Checkpoint / resume.  The noise is a function of (seed, node, time) only
 * (Eqs. (22)-(23) with a counter-based generator), so a run resumed from a
 * checkpoint continues bit-identically to an uninterrupted one.
 * fnlb_checkpoint_bytes: size of the image fnlb_save writes (a small header,
 * the stored populations of every replica as raw stored values, the
 * accumulators).
 * fnlb_save: copies the image into the caller's host buffer of n bytes
 * (FNLB_ENOMEM if smaller); synchronises the stream; returns the watchdog
 * status like the read calls.
 * fnlb_load: restores populations, accumulators, time and sample count from
 * an image made by a handle with the same replicas (parameters and seeds),
 * precision, physics flags and sampling interval, else FNLB_EINVAL (a
 * truncated image: FNLB_ENOMEM).  Synchronises the stream. */
int fnlb_checkpoint_bytes(const fnlb_handle* h, size_t* bytes);
int fnlb_save(fnlb_handle* h, void* host_buf, size_t n);
int fnlb_load(fnlb_handle* h, const void* host_buf, size_t n);

/* Bytes of the device workspace fnlb_sq_misfit_gradient and
 * fnlb_pressure_misfit_gradient need for a horizon
 * of `horizon` steps with populations checkpointed every `ckpt_every` steps:
 * ceil(horizon/ckpt_every) + ckpt_every + 2 state copies plus O(Lx Lz)
 * adjoint fields.  FNLB_EINVAL when the handle does not meet the
 * requirements of fnlb_sq_misfit_gradient (sampling aside). */
int fnlb_adjoint_bytes_required(const fnlb_handle* h, int64_t horizon, int32_t ckpt_every,
                                size_t* bytes);

/* Forward half of fnlb_sq_misfit_gradient: J only.  Runs the forward sweep
 * (populations checkpointed every ckpt_every steps in d_adj) and leaves in
 * d_adj what fnlb_misfit_backward needs to differentiate it.  Requirements,
 * workspace and effects as for fnlb_sq_misfit_gradient. */
int fnlb_sq_misfit(fnlb_handle* h, int32_t field, const double* S_target,
                   const double* weight, int64_t horizon, int32_t ckpt_every,
                   void* d_adj, size_t adj_bytes, double* J);

/* Forward half of fnlb_pressure_misfit_gradient: J only (as fnlb_sq_misfit). */
int fnlb_pressure_misfit(fnlb_handle* h, const double* P_target, const double* weight,
                         int64_t horizon, int32_t ckpt_every, void* d_adj,
                         size_t adj_bytes, double* J);

/* Reverse half: grad = dJ/d(tau_s, tau_d, G) of the last fnlb_sq_misfit or
 * fnlb_pressure_misfit on this handle, by the adjoint sweep over its
 * checkpoints.  d_adj and adj_bytes must be those of that call, its contents
 * untouched, and the handle's time unchanged since (else FNLB_ESTATE;
 * fnlb_reinit and a failed misfit call also end the pairing).  May be called
 * again for the same forward sweep.  Synchronises the stream. */
int fnlb_misfit_backward(fnlb_handle* h, void* d_adj, size_t adj_bytes, double* grad);

/* Vector-Jacobian product of one step of the current state f(t) (Eq. (6)
 * with the collision of Eq. (14), noise of Eqs. (22)-(23) held fixed):
 * given mu_next = dJ/df(t+1), returns mu = (df(t+1)/df(t))^T mu_next and
 * dtheta = mu_next . df(t+1)/d(tau_s, tau_d, G).  mu_next and mu: host
 * arrays in the layout of fnlb_read_populations ([species][l][z][x],
 * 2*9*Lz*Lx doubles); dtheta: 3 doubles.  Requirements as for
 * fnlb_sq_misfit_gradient except sampling (any sample_every); workspace:
 * d_adj of adj_bytes >= fnlb_adjoint_bytes_required(h, 1, 1).  The handle's
 * state and time are unchanged.  Synchronises the stream. */
int fnlb_step_vjp(fnlb_handle* h, const double* mu_next, double* mu, double* dtheta,
                  void* d_adj, size_t adj_bytes);

/* Structure-factor misfit and its gradient by the discrete adjoint of the
 * step, with the noise stream held fixed (the Gaussian variates of every node
 * and step are the same at any parameter value).  From the handle's current
 * state and time, runs `horizon` steps sampling per options.sample_every,
 * forms S(q) = <|Phi|^2> - |<Phi>|^2 of `field` over the half spectrum
 * [k_z][k_x] (k_x = 0..Lx/2) and
 *   J = sum_q weight_q (S(q) - S_target(q))^2,
 * then sweeps the adjoint backwards over checkpointed segments (populations
 * stored every ckpt_every steps and recomputed within a segment) and returns
 * J and grad = dJ/d(tau_s, tau_d, G) (tau_s = 1/lambda_s of Eq. (17),
 * tau_d = 1/lambda_d of Eq. (16), G of Eq. (11)).  Requirements: one replica,
 * FNLB_FP64, options.sample_every > 0, flags FNLB_ASTAR | FNLB_WALL_UZ_FIX,
 * Lx Lz <= 2^20, at least one sample in the horizon.  S_target and weight:
 * host arrays of Lz (Lx/2 + 1) doubles.  d_adj: caller-owned device
 * workspace of adj_bytes >= fnlb_adjoint_bytes_required, 256-byte aligned.
 * The handle's state, time and accumulators are unchanged.  Synchronises
 * the stream. */
int fnlb_sq_misfit_gradient(fnlb_handle* h, int32_t field, const double* S_target,
                            const double* weight, int64_t horizon, int32_t ckpt_every,
                            void* d_adj, size_t adj_bytes, double* J, double* grad);

/* Pressure-profile misfit and its gradient, by the same adjoint: with
 * Pbar_j the time-averaged row mean of P - P_ref over the samples of the
 * horizon (the pressure of fnlb_read_pressure, Eq. (24) / Sec. IV.C),
 *   J = sum_j weight_j (Pbar_j - P_target_j)^2,
 * and grad = dJ/d(tau_s, tau_d, G), G entering both P (its non-local part
 * and P_ref) and the dynamics.  P_target and weight: host arrays of Lz
 * doubles.  Requirements, workspace and effects as for
 * fnlb_sq_misfit_gradient. */
int fnlb_pressure_misfit_gradient(fnlb_handle* h, const double* P_target, const double* weight,
                                  int64_t horizon, int32_t ckpt_every, void* d_adj,
                                  size_t adj_bytes, double* J, double* grad);

/* Frees the handle's host metadata and its streams, events and captured
 * graphs.  Call it once the work enqueued for the handle has finished (for
 * example after a read call, which synchronises).  Caller buffers are
 * untouched. */
int fnlb_destroy(fnlb_handle* h);

/* Static message for an error code. */
const char* fnlb_strerror(int code);

/* Static string identifying the sources the library was built from (a hash
 * of the kernel, runtime and header sources, set by the build), so that a
 * binding can refuse a library older than its sources. */
const char* fnlb_build_id(void);

#ifdef __cplusplus
}
#endif

#endif /* FNLB_H */
