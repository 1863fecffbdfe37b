/*
 * mmcav.h -- C ABI of the MI355X stepper for the Landau-Lifshitz-Gilbert
 * equation on a finite-difference cell grid coupled to N cavity modes
 * (arXiv 2603.03706, "Multimode cavity magnonics in mumax+").
 *
 * What one step computes (all on the GPU, no host round trip per step):
 *   - cavity modes (Sec. II A Eq. (1), Sec. II F Eq. (12); dissipative part
 *     of Sec. IV H Eq. (19) written as a phase Phi_n):
 *         da_n/dt = (-i w_n - k_n) a_n + i g_n e^{-i Phi_n} m^-_n
 *   - mode-weighted co-rotating average (Eq. (2) weighted as in Eq. (18)):
 *         m^-_n = 1/N_geo sum_i G_i u_n(r_i) (1/S) sum_s c_s (m_sx - i m_sy)
 *   - RF feedback along x (Eq. (3), Eq. (13), h0_n = 2 g_n / gamma, Eq. (5)):
 *         B_rf(r) = x c_s sum_n h0_n u_n(r) Re[e^{-i Phi_n} a_n]
 *   - effective field: Zeeman + 6-neighbour exchange (free boundaries) +
 *     uniaxial anisotropy + demag (none | local diagonal | cell-averaged
 *     Newell tensor by zero-padded FFT convolution) + B_rf, and for two
 *     sublattices the intersublattice field -B_E m_{s'}
 *   - Landau-Lifshitz torque with gamma' = gamma / (1 + alpha^2)
 *   - magnetisation and cavity advance inside one Runge-Kutta step
 *     (Sec. III A: the cavity ODEs share the adaptive RK45 step of the LLG
 *     equation): classical RK4 at a fixed step, or Dormand-Prince 5(4) with
 *     a max-norm error over cells and modes; |m| renormalised after each
 *     accepted step.
 *
 * Conventions
 *   - SI units: m, A/m, J/m, J/m^3, T, s; rates w_n, k_n, g_n in rad/s.
 *   - Host arrays are owned by the caller; set_* copy them in, get_* copy
 *     out.  Device memory is owned by the library unless a workspace is
 *     bound (mm_bind_workspace), in which case the caller owns it and must
 *     keep it alive until mm_destroy.
 *   - Cell index i = x + nx (y + ny z); per-sublattice vector fields are
 *     laid out [S][3][nz][ny][nx] (component-major, x fastest).
 *   - Every function returns an mm_status.  No C++ exception crosses the
 *     boundary and the library never aborts.  After an error,
 *     mm_last_error() describes it.  A failed mm_run leaves the state at the
 *     last accepted step.
 *   - One context per thread at a time.  Calls block until their GPU work
 *     has finished.
 */
#ifndef MMCAV_H
#define MMCAV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_ctx mm_ctx;
typedef struct mm_batch mm_batch;

typedef enum {
  MM_OK = 0,
  MM_ERR_ARG = -1,           /* invalid argument (value, size, pointer)      */
  MM_ERR_HIP = -2,           /* HIP runtime error (no device, launch fault)  */
  MM_ERR_OOM = -3,           /* device or host allocation failed             */
  MM_ERR_STATE = -4,         /* call not valid in the current state          */
  MM_ERR_DT_UNDERFLOW = -5,  /* adaptive step fell below dt_min              */
  MM_ERR_NONFINITE = -6      /* state or error estimate became non-finite    */
} mm_status;

enum { MM_DEMAG_NONE = 0, MM_DEMAG_LOCAL = 1, MM_DEMAG_FFT = 2 };
enum { MM_RK4 = 0, MM_DP45 = 1, MM_RK4_SPLIT = 2 };
enum { MM_MAX_MODES = 16 };

typedef struct {
  int32_t nx, ny, nz;          /* grid, each >= 1                              */
  double dx, dy, dz;           /* cell size [m], > 0                           */
  double Ms;                   /* saturation magnetisation per sublattice [A/m] */
  double Aex;                  /* exchange stiffness [J/m]                     */
  double alpha;                /* Gilbert damping, >= 0                        */
  double Ku;                   /* uniaxial anisotropy constant [J/m^3]         */
  double ku_axis[3];           /* anisotropy axis (normalised internally)      */
  double gamma;                /* gyromagnetic ratio [rad/(s T)], e.g. 1.76e11 */
  double B0[3];                /* bias field [T]                               */
  int32_t demag;               /* MM_DEMAG_*                                   */
  double n_local[3];           /* diagonal of the local demag tensor           */
  const uint8_t* geometry;     /* host, nx*ny*nz, nonzero = magnetic; NULL = all */
  int32_t sublattices;         /* 1 (ferromagnet) or 2 (antiferromagnet)       */
  double B_E;                  /* intersublattice exchange field [T] (S = 2)   */
} mm_params;

typedef struct {
  int64_t accepted, rejected;
  double t;                    /* simulated time [s]                           */
  double dt;                   /* current (next proposed) step [s]             */
  double dt_min_seen, dt_max_seen;  /* over accepted steps                     */
  double wall_s;               /* wall time spent in mm_run / mm_batch_run     */
  int32_t status;              /* last run's mm_status                         */
} mm_stats;

/* Create a context for one instance.  Validates the parameters (grid >= 1,
 * nx ny nz sublattices <= 2^26, cells > 0, Ms > 0, gamma > 0, alpha >= 0,
 * demag in range, sublattices in {1, 2}; FFT demag needs sublattices == 1
 * and padded sizes <= 1024) and
 * copies the geometry.  Allocates no device memory.  *out is set only on
 * success. */
mm_status mm_create(const mm_params* p, mm_ctx** out);

/* Release all resources of the context.  NULL is accepted. */
mm_status mm_destroy(mm_ctx* ctx);

/* Device bytes this instance needs for n_modes modes, so a caller can hand
 * over its own memory (e.g. a torch tensor) with mm_bind_workspace. */
mm_status mm_workspace_bytes(const mm_params* p, int32_t n_modes, size_t* bytes);

/* Use caller-owned device memory (at least mm_workspace_bytes for the mode
 * count that mm_set_modes will be given, 256-byte aligned) for all
 * per-instance device buffers.  Must precede the first mm_set_modes. */
mm_status mm_bind_workspace(mm_ctx* ctx, void* device_ptr, size_t bytes);

/* Launch the context's work on this HIP stream (default: a stream owned by
 * the library).  Work submitted by the library waits for work already on
 * the stream and has finished when the call returns. */
mm_status mm_set_stream(mm_ctx* ctx, void* hip_stream);

/* Cavity modes (Sec. II F): n in [0, MM_MAX_MODES]; omega, kappa, g [rad/s]
 * (kappa >= 0); u: host [n][nz][ny][nx] mode profiles, or NULL for u = 1;
 * phi: dissipative phase per mode [rad] or NULL for 0; sublattice_sign:
 * c_s per sublattice (+1/-1) or NULL for +1.  h0_n = 2 g_n / gamma is
 * derived here.  Resets the cavity amplitudes to 0 and the trace. */
mm_status mm_set_modes(mm_ctx* ctx, int32_t n, const double* omega, const double* kappa,
                       const double* g, const float* u, const double* phi,
                       const int8_t* sublattice_sign);

/* Cavity-model variants, per mode (n must equal the mode count; n = 0
 * switches all of them off, as does mm_set_modes):
 *   g_back: backward (cavity-to-magnon) coupling g_b [rad/s] of Sec. II A,
 *     so that the feedback uses h0_n = 2 g_b,n / gamma while the cavity
 *     equation keeps g_n (= g_f); NULL = reciprocal (g_b = g).
 *   kerr: self-Kerr coefficient K_n [rad/s] (Sec. V names Kerr terms as a
 *     cavity-model variant): da_n/dt gains -i K_n |a_n|^2 a_n; NULL = none.
 *   coupling: host [n][n] direct photon-photon coupling J [rad/s], the
 *     H_13 entry of the Sec. II F coupling matrix (Eq. (14)) for any mode pair:
 *     da_n/dt gains -i sum_m J_nm a_m; symmetric with a zero diagonal
 *     (else MM_ERR_ARG); NULL = none.
 * Host arrays, finite values.  The adjoint covers the Kerr term and the
 * mode coupling; mm_run_record and mm_adjoint return MM_ERR_STATE while a
 * backward coupling is set. */
mm_status mm_set_cavity_model(mm_ctx* ctx, int32_t n, const double* g_back, const double* kerr,
                              const double* coupling);

/* Degenerate parametric pump of each mode (Sec. V names parametric drives
 * among the cavity-model variants without giving an equation): da_n/dt
 * gains -i lam_n e^{-2 i wp_n t} conj(a_n), a pump at twice wp_n with
 * complex strength lam_n [rad/s], evaluated at the time of every stage
 * (t + c_s h).  In the frame rotating at wp_n = w_n one quadrature decays at
 * kappa_n + |lam_n| and the other at kappa_n - |lam_n| (parametric gain
 * above the threshold |lam_n| = kappa_n).  lambda: host [n][2] (re, im);
 * omega_p: host [n] wp_n [rad/s]; finite values; n must equal the mode
 * count.  n = 0 or lambda = NULL switches the pump off; mm_set_modes also
 * does.  The adjoint carries the pump's Jacobian. */
mm_status mm_set_parametric(mm_ctx* ctx, int32_t n, const double* lambda, const double* omega_p);

/* External cavity drive eta_n(t) of Eq. (1) / Eq. (12), as the Gaussian
 * pulse of Sec. IV A: eta_n(t) = A_n exp(-((t - t0_n) / sigma_n)^2 / 2),
 * added to da_n/dt at the time of every stage (t + c_s h).  amp: host [n][2]
 * complex amplitude (re, im) [1/s]; t0: pulse centres [s]; sigma: widths
 * [s], > 0, all finite; n must equal the mode count.  n = 0 or amp = NULL
 * switches the drive off.  mm_set_modes also switches it off.  Takes effect
 * from the next run, batched runs included. */
mm_status mm_set_drive(mm_ctx* ctx, int32_t n, const double* amp, const double* t0,
                       const double* sigma);

/* Magnetisation, host [S][3][nz][ny][nx].  Normalised per cell on entry;
 * non-magnetic cells are set to 0.  A magnetic cell with |m| = 0 or a
 * non-finite value is rejected with MM_ERR_ARG. */
mm_status mm_set_m(mm_ctx* ctx, const float* m);

/* Cavity amplitudes, host [n][2] (re, im) in FP64. */
mm_status mm_set_a(mm_ctx* ctx, const double* a);

/* Stepper: method MM_RK4 (fixed step dt0) or MM_DP45 (adaptive, first trial
 * step dt0); dt_min (> 0) ends an adaptive run with MM_ERR_DT_UNDERFLOW when
 * the step would fall below it; dt_max caps the step (<= 0: no cap).
 * MM_RK4_SPLIT is the operator-split co-simulation scheme of Sec. III B, as
 * an accuracy baseline for the joint stepper: per step of dt0 the cavity
 * takes one RK4 step with m^- held at its step-start value, then the LLG
 * takes one RK4 step with the feedback of the new amplitudes held.  It
 * samples like MM_RK4 and has no adjoint (mm_run_record: MM_ERR_STATE). */
mm_status mm_set_stepper(mm_ctx* ctx, int32_t method, double dt0, double dt_min, double dt_max);

/* Record a(t_k) and m^-(t_k) at t_k = t_start + k dt_sample into a device
 * trace of at most max_samples entries, starting at the next run.  DP45:
 * cubic Hermite interpolation over each accepted step.  RK4: dt_sample must
 * be a whole multiple of dt0 (relative slack 1e-9) and samples are step-end
 * values.  max_samples = 0 switches sampling off. */
mm_status mm_set_sampling(mm_ctx* ctx, double dt_sample, int64_t max_samples);

/* Advance by T > 0 seconds.  tol > 0 is the DP45 error tolerance (ignored
 * for RK4).  The last step is clipped to land on t + T.  Returns MM_OK,
 * MM_ERR_DT_UNDERFLOW or MM_ERR_NONFINITE (state kept at the last accepted
 * step), or an argument/HIP error. */
mm_status mm_run(mm_ctx* ctx, double T, double tol);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mm_run with
 * the same arguments, semantics and arithmetic (bit for bit the result of
 * mm_run with its default FFT choices), whose per-run scratch -- stage
 * derivatives and inputs, workgroup partial records, the demag field and
 * spectra, the instance descriptor, work tables and done flags -- lives in a
 * fixed static device array of MM_NOALLOC_SCRATCH_BYTES (every GPU the
 * library runs on holds its own copy until the process ends) instead of
 * memory the library allocates.  The call makes no hipMalloc, hipFree, pinned-memory or
 * stream/graph creation call; it launches eagerly on the context's stream
 * (mm_set_stream; the null stream if none) and waits for the run.  The
 * context must be set up (mm_set_modes and mm_set_m, which allocate its
 * state).  MM_ERR_ARG if the instance's scratch exceeds the array (about
 * 108 B per cell and sublattice plus, with FFT demag, 12 B per cell and the
 * x-transformed rows: e.g. a 64^3 grid with FFT demag fits, a 128x128x32 one
 * does not).  The array is cleared where it must start at zero at every
 * call.  Runs of one process on one GPU share its array and are serialised
 * by a lock; runs on one GPU that overlap from two processes each have their
 * own array. */
#define MM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
mm_status mm_run_noalloc(mm_ctx* ctx, double T, double tol);

/* Copy out m [S][3][nz][ny][nx] (FP32) and a [n][2] (FP64). */
mm_status mm_get_m(const mm_ctx* ctx, float* out);
mm_status mm_get_a(const mm_ctx* ctx, double* out);

/* Copy out the trace: t [n], a [n][modes][2], mminus [n][modes][2]; *n is
 * in: capacity, out: samples recorded. */
mm_status mm_get_trace(const mm_ctx* ctx, double* t, double* a, double* mminus, int64_t* n);

mm_status mm_get_stats(const mm_ctx* ctx, mm_stats* out);

/* Checkpoint / resume: serialise (m, a, t, dt, counters) into blob.  Call
 * with blob = NULL to query *bytes. */
mm_status mm_get_state(const mm_ctx* ctx, void* blob, size_t* bytes);
mm_status mm_set_state(mm_ctx* ctx, const void* blob, size_t bytes);

/* ---- batched form: many instances stepped together ------------------- */
/* Group count >= 1 contexts (all with modes set and the same method).  The
 * contexts stay owned by the caller and must outlive the batch.  Each
 * instance keeps its own t, dt, status and trace; one launch sequence
 * (captured in a HIP graph) advances all of them.  The batch may instead
 * run as sub-batches of about equal cell count, each with its own stream and
 * graphs, whose launch sequences the device runs concurrently, so that the
 * last, partly filled round of workgroups of one kernel overlaps another
 * part's next kernel (mm_batch_set_streams, or chosen by timing in
 * mm_batch_tune).  An instance's arithmetic does not depend on the split. */
mm_status mm_batch_create(mm_ctx* const* ctxs, int32_t count, mm_batch** out);
/* Re-split the batch into `parts` sub-batches (1..8, at most the instance
 * count; 1 = one launch sequence for all).  Waits for the batch's streams;
 * FFT strategy choices (mm_batch_tune, mm_batch_set_fft_*) return to their
 * defaults.  The handle stays valid.  MM_ERR_ARG for parts out of range. */
mm_status mm_batch_set_streams(mm_batch* b, int32_t parts);
/* Number of sub-batches the batch runs as. */
mm_status mm_batch_get_streams(const mm_batch* b, int32_t* parts);
/* Advance every instance by T (tol as in mm_run).  Returns the first
 * non-OK instance status, or MM_OK; per-instance status in mm_get_stats. */
mm_status mm_batch_run(mm_batch* b, double T, double tol);
/* Advance every unfinished instance by exactly `steps` attempted steps from
 * its current state (t_end = +inf), for throughput measurement.  The run
 * starts by evaluating the first derivative at the current state (as every
 * run does) and ends by reading each instance's statistics back; the steps
 * run as captured graphs (32-step graphs, then graphs of 16, 8, 4, 2 and 1
 * steps for the remainder). */
mm_status mm_batch_step(mm_batch* b, int64_t steps, double tol);
mm_status mm_batch_destroy(mm_batch* b);

/* Open-ended stepping in three calls, so that a caller can time or stream
 * steps without the per-run set-up and read-back (Sec. III A: the RK45 loop
 * stays on the device with no per-step host transfer):
 *  - mm_batch_begin sets every instance's run parameters (no end time, tol
 *    as in mm_run), enqueues the run-start derivative and captures every
 *    step graph; it returns without waiting for the device.
 *  - mm_batch_advance enqueues exactly `steps` further attempted steps of
 *    every unfinished instance as graph launches on the batch's streams and
 *    returns at once; consecutive calls continue one run (FSAL, dt and the
 *    trace carry over), bit for bit as one mm_batch_step of the summed count.
 *  - mm_batch_end waits for the device, reads every instance's statistics
 *    (mm_get_stats) and returns the first non-OK instance status.
 * Between begin and end, any call on the batch or on one of its contexts
 * other than advance, end and mm_batch_destroy (which waits and closes the
 * run) returns MM_ERR_STATE; so does begin on a batch with an open run or
 * with an instance in another open run, and advance/end with none. */
mm_status mm_batch_begin(mm_batch* b, double tol);
mm_status mm_batch_advance(mm_batch* b, int64_t steps);
mm_status mm_batch_end(mm_batch* b);

/* Accepted and rejected step counts summed over the batch's instances, as
 * they stand once the work enqueued so far has finished (the call waits for
 * the batch's streams).  Read only, so it is allowed during an open run,
 * e.g. between two mm_batch_advance calls; the counts are cumulative over
 * every run of the instances, as in mm_get_stats.  NULL outputs are
 * skipped. */
mm_status mm_batch_counts(mm_batch* b, int64_t* accepted, int64_t* rejected);

/* Autotune the batch.  With two or more instances it first times whole
 * steps (32 + 2 x 64 attempted steps) of the batch run as 1, 2 and 3
 * concurrent sub-batches (mm_batch_set_streams) and keeps the fastest; then,
 * in every sub-batch, the demag FFT of every grid shape: the x passes for
 * each tile width and the y-z work either fused in one LDS-resident kernel or
 * split into y / z passes for each tile shape, keeping the fastest.  Every
 * instance's state (and trace, counters, statistics) is left as it was.  A
 * JSON list of the choices and timings, one entry per grid shape and
 * sub-batch ("part": its index), is written to report (may be NULL). */
mm_status mm_batch_tune(mm_batch* b, char* report, size_t report_len);
/* The FFT part of mm_batch_tune only: the batch keeps its sub-batch count. */
mm_status mm_batch_tune_fft(mm_batch* b, char* report, size_t report_len);

/* Demag y-z strategy for every FFT grid shape in the batch (mm_batch_tune
 * chooses one per shape by timing; before that the exchange strategy is used
 * where it applies, else the eight-lane register one, else the register one,
 * else the fused one where it fits, else the split exchange one, else the
 * split one):
 *   MM_YZ_FUSED     y and z lines transformed in LDS by one workgroup per
 *                   (instance, kx), z in tiles of ky columns;
 *   MM_YZ_REGISTER  one workgroup per (instance, kx), each line split over
 *                   four lanes that hold it in registers; padded y of 16..128
 *                   and padded z of 16..64 cells only;
 *   MM_YZ_SPLIT     separate y and z passes through device memory;
 *   MM_YZ_REGISTER8 as MM_YZ_REGISTER with each z line over eight lanes
 *                   (half the registers per lane); padded z of 32 or 64;
 *   MM_YZ_EXCHANGE  one workgroup per (instance, kx), each line over 2..8
 *                   lanes in two register passes joined by one exchange
 *                   through LDS; padded y of 16..128, padded z of 32 or 64.
 *   MM_YZ_SPLIT_EXCHANGE  the split passes with the y passes done by the
 *                   line transforms of MM_YZ_EXCHANGE (whole rows per lane
 *                   group) and the z pass of MM_YZ_SPLIT; padded y of 16..256.
 * All of them compute the same convolution (agreement to FP32 rounding).
 * Returns MM_ERR_ARG, changing nothing, if some shape cannot use `path`. */
enum {
  MM_YZ_FUSED = 0,
  MM_YZ_REGISTER = 1,
  MM_YZ_SPLIT = 2,
  MM_YZ_REGISTER8 = 3,
  MM_YZ_EXCHANGE = 4,
  MM_YZ_SPLIT_EXCHANGE = 5
};
mm_status mm_batch_set_fft_path(mm_batch* b, int32_t path);

/* Strategy of the x passes (R2C forward, C2R inverse) for every FFT grid
 * shape: MM_X_STAGE (the default where it applies: nx a power of two from 2
 * to 256, one sublattice) does them inside the stage kernels, each workgroup
 * for its own whole x-rows, so the demag field never goes through device
 * memory and the next stage input is transformed where it is computed;
 * MM_X_LDS transforms tiles of rows in separate kernels; MM_X_REGISTER does
 * so with each pair of real rows as one complex line over four lanes in
 * registers (padded x of 16..128 cells only).  Same results to FP32
 * rounding.  MM_ERR_ARG, changing nothing, if a shape cannot use `path`. */
enum { MM_X_LDS = 0, MM_X_REGISTER = 1, MM_X_STAGE = 2 };
mm_status mm_batch_set_fft_x(mm_batch* b, int32_t path);

/* Per-kernel timing: run `steps` steps eagerly, timing each launch with HIP
 * events on the library stream (for a split batch: the whole batch as one
 * launch sequence with the FFT strategies of its first part, each kernel
 * alone on the device).  Fills up to `cap` entries: names (each
 * char[48]), launches, total milliseconds, algorithmic bytes per launch
 * (the bytes a launch must read and write; see the kernel notes).  *n is
 * set to the number of kernel kinds. */
mm_status mm_batch_profile(mm_batch* b, int64_t steps, double tol, int32_t cap, char* names,
                           int64_t* launches, double* total_ms, double* bytes_per_launch, int32_t* n);

/* ---- form (3): discrete adjoint (fixed-step RK4 runs; adaptive DP45 runs by replay) */
/* Advance by T (a whole number of RK4 steps of dt0, relative slack 1e-9)
 * from the current state and keep a checkpoint (m, a, t) every
 * `checkpoint_every` steps (device memory) for a later mm_adjoint.  The
 * context must use MM_RK4 (not MM_RK4_SPLIT) and reciprocal coupling (no
 * g_back from mm_set_cavity_model), else MM_ERR_STATE; the drive, the Kerr
 * term and the mode coupling are covered.  Replaces any earlier recording.
 * With sampling set (dt_sample = dt0), the trace of the recorded run gives
 * a at every step end for mm_adjoint_trace. */
mm_status mm_run_record(mm_ctx* ctx, double T, int32_t checkpoint_every);

/* Adjoint of adaptive runs (form (3) for the DP45 stepper): advance by T
 * with DP45 at tolerance tol (as mm_run) from the current state, keeping the
 * size of every accepted step, then replay the accepted steps from the
 * start (each at its logged size, all accepted: rejected attempts leave no
 * trace in the state, so the replay reaches the run's states bit for bit)
 * and keep a checkpoint every `checkpoint_every` accepted steps.  A later
 * mm_adjoint differentiates that replayed map, the step sizes held fixed --
 * the usual adjoint of an adaptive run.  The context must use MM_DP45 and
 * reciprocal coupling, else MM_ERR_STATE; losses on the trace
 * (mm_adjoint_trace) are built for RK4 runs only.  The state is left at the
 * end of the run with its own controller state, counters and trace.
 * Device memory: the step log (8 B per accepted step) and the checkpoints;
 * mm_adjoint then keeps six stage inputs per step of a segment. */
mm_status mm_run_record_adaptive(mm_ctx* ctx, double T, double tol, int32_t checkpoint_every);
/* Sizes of the accepted steps of the last mm_run_record_adaptive, negative
 * for the last one when it was clipped onto the end time: *n is in: the
 * capacity of h (may be 0 with h = NULL), out: the number of steps. */
mm_status mm_get_step_log(const mm_ctx* ctx, double* h, int64_t* n);

/* Gradients of a scalar loss L(m(T), a(T)) of the recorded run, by the
 * discrete adjoint of the recorded step sequence (each segment between
 * checkpoints is recomputed with its stage inputs, and with FFT demag their
 * demag fields, kept on the device, then reversed stage by stage).  Inputs: dL_da [n][2] = (dL/dRe a_n, dL/dIm a_n)
 * at T (required); dL_dm [S][3][nz][ny][nx] at T or NULL (zero).  Outputs
 * (each may be NULL): grad_u [n][nz][ny][nx] (d L / d u_n(r), also for
 * modes set without a profile, i.e. at u = 1), grad_g [n], grad_alpha [1],
 * grad_B0 [3], grad_a0 [n][2] and grad_m0 [S][3][nz][ny][nx] (with respect
 * to the normalised initial state).  The context's state is left at the end
 * of the recorded run.  Device memory: 4 (K+1) + 5 state-sized buffers
 * (plus 4 K field-sized ones with FFT demag) for K = checkpoint_every, plus
 * the checkpoints. */
mm_status mm_adjoint(mm_ctx* ctx, const double* dL_da, const float* dL_dm, float* grad_u, double* grad_g,
                     double* grad_alpha, double* grad_B0, double* grad_a0, float* grad_m0);

/* As mm_adjoint, for a loss that also depends on the cavity trace of the
 * recorded run, L(a(t_0), a(t_1), ..., a(t_K), m(T)) with t_k = t_0 + k dt
 * the step ends (spectral objectives such as |sum_k a(t_k) e^{i w t_k}|^2,
 * the observable of Sec. IV).  dL_dtrace: host [count][n][2] =
 * (dL/dRe a_n(t_k), dL/dIm a_n(t_k)), count = recorded steps + 1 (else
 * MM_ERR_ARG); each entry is added to the cavity adjoint when the reverse
 * pass reaches its step end, entry 0 to grad_a0.  dL_da (a further
 * derivative at T) may be NULL.  The buffer is copied to the device for the
 * call (count * n * 16 bytes) and freed before it returns. */
mm_status mm_adjoint_trace(mm_ctx* ctx, const double* dL_dtrace, int64_t count, const double* dL_da,
                           const float* dL_dm, float* grad_u, double* grad_g, double* grad_alpha,
                           double* grad_B0, double* grad_a0, float* grad_m0);

/* ---- host-side checks (no GPU needed) ------------------------------------ */
/* Cell-averaged demag tensor (xx, yy, zz, xy, xz, yz) at displacement
 * (X, Y, Z) [m] for cells dx*dy*dz, as the library's setup computes it. */
mm_status mm_demag_tensor(double X, double Y, double Z, double dx, double dy, double dz,
                          double* out6);

/* Description of the last error on this thread (never NULL).  The error
 * text is kept per calling thread rather than per context: every entry point
 * (including mm_create, which has no context yet, and the batch calls, which
 * span several) records its failure in the same place, and with one context
 * per thread at a time the two are the same. */
const char* mm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MMCAV_H */
