/*
 * nmfa.h -- C ABI of the MI355X (gfx950) noisy mean-field annealing library (libnmfa.so).
 *
 * Noisy mean-field annealing (NMFA) is the method of A. D. King, W. Bernoudy, J. King,
 * A. J. Berkley, T. Lanting, "Emulating the coherent Ising machine with a mean-field algorithm"
 * (arXiv:1806.08422, Sec. II, Alg. 1). For an Ising problem (h, J) it anneals a continuous state
 * s in [-1, 1]^N from s = 0 over t = 1..t_f iterations of a decreasing temperature T_t. One
 * iteration replaces every component at once by a damped Boltzmann expectation in the noisy,
 * normalised mean field:
 *
 *   s_i <- alpha * ( -tanh( [ (h_i + (J s)_i) / sqrt(h_i^2 + sum_j J_ij^2) + sigma z_i ] / T_t ) )
 *          + (1 - alpha) * s_i,            z_i ~ N(0, 1) independently for every (t, replica, i),
 *
 * and the sample is the sign of the final state. This library runs R independent samples
 * ("replicas") at once on one GPU and evaluates the Ising energy of Eq. 1,
 * H = sum_{i<j} J_ij s_i s_j + sum_i h_i s_i, of each sample.
 *
 * Conventions shared by every entry point:
 *   - Every call returns an int status: NMFA_OK (0) or a negative NMFA_E* code. A failing call
 *     leaves a message retrievable with nmfa_last_error() (thread-local) and never aborts.
 *   - Matrices are dense, row-major, with the given leading dimension n. Pointers are HOST
 *     pointers unless the argument says "device". The caller owns every buffer it passes in;
 *     the library deep-copies what it keeps.
 *   - Noise: Philox4x32-10 (Salmon et al., SC'11) keyed by the 64-bit seed (low word first), with
 *     counter (floor(i/4), r, t, 0) for spin i of replica r at iteration t (1-based). Its four
 *     output words give four uniforms and Box-Muller turns (u0,u1), (u2,u3) into the Gaussians
 *     of spins 4q..4q+3. Replica r's noise does not depend on R, so replica r of any run with
 *     the same seed, instance and parameters sees the same noise.
 *   - Temperature schedule (the paper's Fig. 2 is a three-segment piecewise-exponential
 *     schedule whose values are not printed): knots (u_k, T_k), u_0 = 0 < ... < u_K = 1, log T
 *     linear between knots, T_t = T((t-1)/(t_f-1)). The default knots are
 *     (0, 10) (0.1, 2) (0.6, 0.5) (1, 0.05). A caller may instead pass the temperatures
 *     T_1..T_tf themselves (nmfa_params.T_explicit).
 */
#ifndef NMFA_H
#define NMFA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------------------------- */
#define NMFA_OK 0
#define NMFA_EINVAL (-1)    /* invalid argument (sizes, non-symmetric J, NaN, bad schedule...) */
#define NMFA_ENOMEM (-2)    /* device or host allocation failed, or a budget is exceeded */
#define NMFA_EDEVICE (-3)   /* a HIP runtime call failed (message names it) */
#define NMFA_ESTATE (-4)    /* call out of order, e.g. spins requested before any anneal */
#define NMFA_ECANCELED (-5) /* serving: the request was cancelled */

/* ---- precisions ------------------------------------------------------------------------------
 * NMFA_FP64       J, S and all epilogue arithmetic in FP64 (validation path; FP64 MFMA).
 * NMFA_FP32       J and S in FP32 on FP32 MFMA; normalisation, noise, tanh and state in FP32.
 * NMFA_BF16       J and S rounded to BF16 on BF16 MFMA with FP32 accumulation; FP32 epilogue and
 *                 FP32 master state (S is a BF16 copy of the FP32 state).
 * NMFA_FP8J_BF16S J stored as FP8 E4M3 (exact for integers |J| <= 16), widened to BF16 for the
 *                 MFMA; spins as in NMFA_BF16.
 * NMFA_FP8J_FP8S  J rounded to FP8 E4M3 as for NMFA_FP8J_BF16S and the spin operands rounded to
 *                 FP8 E4M3 (nearest even): the mean field is an FP4 (J) x FP8 (spins) matrix
 *                 product with FP32 accumulation; FP32 epilogue and master state. Only for
 *                 couplings that FP4 E2M1 holds exactly (e.g. {0, +-1}) and n <= 2048 (the
 *                 register-J kernel, paths 4/5); nmfa_create fails with NMFA_EINVAL otherwise.
 * J values that the chosen storage type cannot represent are rounded to nearest; the energies
 * are always computed from the exact couplings given to nmfa_create. */
typedef enum nmfa_precision {
  NMFA_FP64 = 0,
  NMFA_FP32 = 1,
  NMFA_BF16 = 2,
  NMFA_FP8J_BF16S = 3,
  NMFA_FP8J_FP8S = 4
} nmfa_precision;

/* ---- flags ------------------------------------------------------------------------------------ */
#define NMFA_FLAG_NEGATE_NOISE 0x1u   /* test hook: use -z for every Gaussian z */
#define NMFA_FLAG_UPPER_TRIANGULAR 0x2u /* J holds only i<j; the library mirrors it */
#define NMFA_FLAG_FORCE_STEP 0x4u     /* use the per-iteration (large-N) kernel even if N is small */
#define NMFA_FLAG_FORCE_XCD 0x8u      /* use the persistent XCD-group kernel (BF16 / FP8-J only) */
#define NMFA_FLAG_FORCE_FENCED 0x10u  /* XCD-group kernel: exchange with device-scope fences */
#define NMFA_FLAG_FORCE_LDS_J 0x20u   /* XCD-group kernel: keep J in LDS even where the
                                         register-resident variant applies (test hook) */
#define NMFA_FLAG_FORCE_SPARSE 0x40u  /* use the sparse (ELL) kernel: at most 64 couplings per row */
#define NMFA_FLAG_SPARSE_GENERIC 0x80u /* sparse kernel: read the couplings from global memory every
                                         iteration even where the register variant applies (test hook) */

/* ---- parameters ------------------------------------------------------------------------------
 * Fill with nmfa_params_default() and override fields. struct_size must be sizeof(nmfa_params)
 * (ABI versioning). Pointers inside are read during nmfa_create only. */
typedef struct nmfa_params {
  uint32_t struct_size;
  uint32_t precision;      /* nmfa_precision */
  double alpha;            /* damping, 0 < alpha <= 1; paper: 0.15 (Sec. II) */
  double sigma;            /* noise standard deviation, >= 0; paper: 0.15 (Sec. II) */
  int32_t n_knots;         /* 0: default schedule; else number of (knot_u, knot_T) pairs */
  const double *knot_u;    /* n_knots increasing values, first 0 and last 1 (if n_knots > 1) */
  const double *knot_T;    /* n_knots temperatures > 0 */
  uint32_t flags;          /* NMFA_FLAG_* */
  int32_t record_iters;    /* keep s after each of the first record_iters iterations */
  int32_t n_T_explicit;    /* 0: temperatures from the knots. Else the schedule is given point by
                              point: T_t = T_explicit[t-1] for t = 1..n_T_explicit (the knots are
                              ignored), and every anneal of the context must use t_f = n_T_explicit
                              (others fail with NMFA_EINVAL) */
  const double *T_explicit; /* n_T_explicit finite temperatures > 0 (host; copied at create) */
} nmfa_params;

typedef struct nmfa_ctx nmfa_ctx;

/* Defaults: alpha = sigma = 0.15, default schedule (no explicit temperatures), NMFA_BF16, no
 * flags, no recording. */
void nmfa_params_default(nmfa_params *p);

/* Create a solver for the instance (h, J) (Eq. 1; Alg. 1 inputs).
 *   n      number of spins, 1 <= n <= 16384
 *   J      host, n*n doubles: symmetric with zero diagonal (or the upper triangle with
 *          NMFA_FLAG_UPPER_TRIANGULAR), finite
 *   h      host, n doubles, or NULL for h = 0
 *   p      parameters (NULL: defaults)
 *   out    receives the handle; release it with nmfa_destroy
 * Computes the normalisers sqrt(h_i^2 + sum_j J_ij^2) in FP64 (a zero normaliser makes that
 * spin's field term 0), converts J to the precision's storage type and uploads everything to
 * the current HIP device. Errors: EINVAL, ENOMEM, EDEVICE. */
int nmfa_create(int32_t n, const double *J, const double *h, const nmfa_params *p, nmfa_ctx **out);

/* Run the whole anneal: iterations 1..t_f of Algorithm 1 on R replicas, then the sign readout
 * and the energies of all R samples, enqueued on `hip_stream` (a hipStream_t; NULL = the null
 * stream). Asynchronous: returns after enqueueing; results are read with nmfa_spins /
 * nmfa_energies, which synchronise. Device buffers are (re)allocated only when R grows.
 * A call may be recorded into a HIP graph on a capturing stream once an earlier call with the
 * same R and t_f has run eagerly (that call allocates the run buffers and uploads the schedule;
 * a recorded call enqueues kernels and event records only); replaying the graph repeats the
 * recorded call exactly, seed included.
 * Errors: EINVAL (R < 1, t_f < 1, t_f other than n_T_explicit when explicit temperatures
 * were given), ENOMEM, EDEVICE. */
int nmfa_anneal(nmfa_ctx *c, int32_t R, int32_t t_f, uint64_t seed, void *hip_stream);

/* Checkpoint/resume form: run iterations t_begin..t_end (1 <= t_begin <= t_end <= t_f) of a
 * t_f-iteration schedule. t_begin = 1 starts from s = 0; t_begin > 1 continues from the state
 * the previous call left (same R, t_f, seed) or from nmfa_set_state. The readout and energies
 * are recomputed after every call. Errors: EINVAL, ESTATE (no state to continue), ENOMEM, EDEVICE. */
int nmfa_anneal_range(nmfa_ctx *c, int32_t R, int32_t t_f, int32_t t_begin, int32_t t_end,
                      uint64_t seed, void *hip_stream);

/* Copy the R*n readout spins s~ (+1/-1, replica-major) to `out` (host, or device if on_device).
 * Synchronises the anneal's stream. Errors: ESTATE, EDEVICE. */
int nmfa_spins(nmfa_ctx *c, int8_t *out, int32_t on_device);

/* Copy the R energies H(s~) (Eq. 1 over pairs i<j) to E (host, R doubles). If J and h are
 * integral (and max|J_ij| * n^2 < 2^52, so that every partial sum is exact), E_int (host, R int64,
 * or NULL) receives the exact integer energies; otherwise E_int is filled with 0. Synchronises.
 * On the group-kernel paths (2-5) every call that reads results or state also checks the kernels'
 * abort word, also after a run replayed from a recorded HIP graph. Errors: ESTATE, EDEVICE (a HIP
 * call failed, or a group barrier of the run timed out). */
int nmfa_energies(nmfa_ctx *c, double *E, int64_t *E_int);

/* MAX-CUT values (Table I convention, J = edge weights, h = 0): cut_r = (sum_{i<j} J_ij - H_r)/2.
 * Host, R doubles. Errors: ESTATE, EDEVICE. */
int nmfa_cuts(nmfa_ctx *c, double *cut);

/* Energies (and exact integer energies if J, h are integral) of R caller-supplied spin vectors
 * (host, R*n int8 of +1/-1). Synchronous. Errors: EINVAL, ENOMEM, EDEVICE. */
int nmfa_energies_of(nmfa_ctx *c, int32_t R, const int8_t *spins, double *E, int64_t *E_int);

/* The same energies as nmfa_energies_of, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): it calls no
 * hipMalloc, hipFree or allocating library routine. Inputs and outputs are DEVICE pointers the
 * caller owns: d_spins R*n int8 (+1/-1, replica-major; not checked: other values are used as the
 * integers they are), d_E R doubles, d_E_int R int64 or NULL (0 unless the energies are exact
 * integers, as for nmfa_energies_of). Asynchronous on hip_stream (NULL = null stream): the
 * results are ready when the stream reaches them. Where the context keeps the int8 copy of J
 * (integral |J| <= 127) the kernels take their scratch -- the zero-padded signs,
 * roundup(R, 64) * roundup(n, 64) bytes rounded up to 256, and R 64-bit partial sums -- from a
 * fixed device array of NMFA_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; larger
 * requests fail with NMFA_EINVAL. Every call on one GPU shares that array, so calls that overlap
 * on one GPU (other streams, other threads) race and must be serialised by the caller.
 * Errors: EINVAL (NULL pointer, R < 1, scratch too small), EDEVICE. */
#define NMFA_NOALLOC_SCRATCH_BYTES (16u << 20)
int nmfa_energies_of_noalloc(nmfa_ctx *c, int32_t R, const int8_t *d_spins, double *d_E, int64_t *d_E_int,
                             void *hip_stream);

/* Continuous state s after the last call (host, R*n doubles, widened from FP32 on the FP32/BF16
 * paths). Synchronises. Errors: ESTATE, EDEVICE. */
int nmfa_get_state(nmfa_ctx *c, double *out);

/* Replace the continuous state (host, R*n doubles, rounded to the master precision), e.g. to
 * resume from a checkpoint with nmfa_anneal_range(t_begin > 1). Errors: EINVAL, ENOMEM, EDEVICE. */
int nmfa_set_state(nmfa_ctx *c, int32_t R, const double *in);

/* Trajectory of the last call: out[(k*R + r)*n + i] = s_i of replica r after its k-th iteration,
 * k < min(record_iters, iterations run) (host, doubles). Errors: ESTATE, EDEVICE. */
int nmfa_trajectory(nmfa_ctx *c, double *out);

/* Information about a context: writes n, the precision and the kernel path (0 = persistent
 * small-N kernel with J in LDS; 1 = per-iteration kernel; 2 = persistent XCD-group kernel with
 * J rows in LDS whose groups exchanged spins through one XCD's L2; 3 = the same kernel with
 * device-scope fences, used when a group's workgroups were not all placed on one XCD; 4 and 5 =
 * the XCD-group kernel with J rows held in registers (FP4-exact couplings, n <= 2048), exchange
 * as for 2 and 3; 6 = the sparse kernel, J as nonzeros per row (chosen for n > 256 when every
 * row has at most min(64, n/8) couplings and either the register variant below applies or no
 * XCD-group kernel does, or with NMFA_FLAG_FORCE_SPARSE); 7 = the sparse kernel with each
 * thread's rows of J held in registers (at most 16 couplings per row, n <= 4096, fewer
 * couplings per row above n = 2048).
 * Paths 2/3, 4/5 and 6/7 are only told apart after an anneal has completed (the call
 * synchronises). Errors: EINVAL, EDEVICE. */
int nmfa_info(nmfa_ctx *c, int32_t *n, int32_t *precision, int32_t *path);

/* Storage format of J in device memory as the annealing kernel reads it. For the BF16-operand
 * precisions on the group and per-iteration kernels J (already rounded as the precision
 * prescribes, Sec. III) is kept in the narrowest of these formats that holds every coupling
 * exactly and is widened to BF16 in registers: NMFA_JFMT_BF16, NMFA_JFMT_FP8 (E4M3),
 * NMFA_JFMT_FP4 (E2M1); the small-N kernel keeps BF16 (FP8 for NMFA_FP8J_BF16S).
 * NMFA_JFMT_NATIVE: J in the precision's own type (FP64, FP32). Errors: EINVAL. */
#define NMFA_JFMT_BF16 0
#define NMFA_JFMT_FP8 1
#define NMFA_JFMT_FP4 2
#define NMFA_JFMT_NATIVE 3
#define NMFA_JFMT_ELL 4 /* sparse kernel: nonzeros per row with column indices, FP32 (FP64 for FP64) */
int nmfa_j_format(nmfa_ctx *c, int32_t *fmt);

/* Device time of the last anneal in milliseconds, from HIP events recorded on the anneal's own
 * stream: *anneal_ms covers the annealing kernel launches only (Algorithm 1's iterations),
 * *total_ms also the readout and the energy evaluation; *launches is the number of annealing
 * kernel launches (1 for the persistent kernels, one per iteration for the per-iteration path).
 * Any output pointer may be NULL. Synchronises. Errors: ESTATE, EDEVICE. */
int nmfa_last_timing(nmfa_ctx *c, double *anneal_ms, double *total_ms, int32_t *launches);

/* Test hook for the group-kernel paths (2-5): sets the kernels' abort word as a group barrier
 * that timed out would, so that a caller can check that the next read of results or state
 * reports NMFA_EDEVICE. nmfa_set_state and the next anneal from t = 1 clear it.
 * Errors: EINVAL (not a group-kernel context), EDEVICE. */
int nmfa_debug_raise_abort(nmfa_ctx *c);

/* Release every device and host resource of the context (NULL is ignored). */
void nmfa_destroy(nmfa_ctx *c);

/* ---- noise stream utilities (the generator the anneal uses, exposed for reproducibility) ----
 * nmfa_noise_words: the Philox4x32-10 output words for counters (q, r0+k, t, 0), k < n_rep,
 *   q < n_quads: out[4*(k*n_quads + q) + w] (host, 4*n_rep*n_quads uint32).
 * nmfa_noise_values: the corresponding standard normal numbers z(t, r0+k, 4q+w) as the FP64
 *   path (fp64 = 1) or the FP32 paths (fp64 = 0) compute them, widened to double.
 * Synchronous. Errors: EINVAL, ENOMEM, EDEVICE. */
int nmfa_noise_words(uint64_t seed, int32_t t, int32_t r0, int32_t n_rep, int32_t n_quads, uint32_t *out);
int nmfa_noise_values(uint64_t seed, int32_t t, int32_t r0, int32_t n_rep, int32_t n_quads, int32_t fp64,
                      double *out);

/* Human-readable message of the last failing call on this thread ("" if none). */
const char *nmfa_last_error(void);

/* ---- serving: continuous batching of annealing requests ---------------------------------------
 * A server owns three GPU streams, a scheduler thread and an admission thread. Requests
 * (instance, R, t_f, seed) are admitted in arrival order while the device memory they need fits
 * in hbm_budget_bytes and fewer than max_active are running; a request that does not fit waits
 * (later requests do not overtake it), one larger than the whole budget fails with NMFA_ENOMEM.
 * The admission thread does each admitted request's host-side set-up and upload while the device
 * runs. Admitted requests are advanced in rounds of chunk_iters iterations: every round runs one
 * batched launch of the persistent small-N kernel over the replica blocks of all admitted small-N
 * requests, plus the large-N requests' own kernels side by side on the other streams, and the
 * next round is enqueued before the previous one is waited for; requests that arrive while others
 * run join at a following round. J and the spin state stay on the device between rounds. A
 * finished request's device memory is freed in batches (or when admission needs it), so
 * bytes_in_use can stay above the running requests' needs for a while. Because the
 * noise is counter-based and every request's arithmetic depends only on that request, a
 * request's result is bit-identical alone and in any mix. The scheduler runs the paper's
 * Algorithm 1 per request exactly as nmfa_anneal does (same kernels, same precision). */
typedef struct nmfa_server nmfa_server;

typedef struct nmfa_server_params {
  uint32_t struct_size;       /* sizeof(nmfa_server_params) */
  uint32_t precision;         /* nmfa_precision of every request; default NMFA_BF16 */
  uint64_t hbm_budget_bytes;  /* device memory the admitted requests may hold; default 8 GiB */
  int32_t max_active;         /* admitted requests at once; default 256 */
  int32_t chunk_iters;        /* iterations per scheduling round; default 250 */
} nmfa_server_params;

typedef struct nmfa_server_stats {
  uint64_t submitted, completed, failed, cancelled;
  uint64_t queued, active;            /* at the time of the call */
  uint64_t bytes_in_use, peak_bytes;  /* admitted, not yet freed device bytes (the budget's accounting) */
  uint64_t rounds, batched_launches;
} nmfa_server_stats;

/* Request states reported by nmfa_server_poll. */
#define NMFA_JOB_QUEUED 0
#define NMFA_JOB_RUNNING 1
#define NMFA_JOB_DONE 2

void nmfa_server_params_default(nmfa_server_params *p);

/* Start a server on the current HIP device. Errors: EINVAL, ENOMEM, EDEVICE. */
int nmfa_server_create(const nmfa_server_params *p, nmfa_server **out);

/* Queue a request: n spins, J (host, n*n, symmetric, zero diagonal), h (host, n, or NULL),
 * R replicas, t_f iterations, noise seed. The library copies J and h before returning; the
 * instance is validated when the request is admitted (a bad instance fails the request).
 * *ticket identifies the request. Errors: EINVAL (sizes), ESTATE (server stopping). */
int nmfa_server_submit(nmfa_server *s, int32_t n, const double *J, const double *h, int32_t R, int32_t t_f,
                       uint64_t seed, uint64_t *ticket);

/* *status = NMFA_JOB_QUEUED / RUNNING / DONE, or the negative error code of a failed or
 * cancelled (NMFA_ECANCELED) request. Errors: EINVAL (unknown ticket). */
int nmfa_server_poll(nmfa_server *s, uint64_t ticket, int32_t *status);

/* Block until the request has finished (done, failed or cancelled) or timeout_ms elapsed
 * (negative: no limit). Returns NMFA_OK when it finished, NMFA_ESTATE on timeout. */
int nmfa_server_wait(nmfa_server *s, uint64_t ticket, int32_t timeout_ms);

/* Results of a finished request: E (R doubles), E_int (R int64, or NULL; 0 unless J and h are
 * integral), spins (R*n int8, or NULL), latency_ms (submit to results on the host, or NULL).
 * Errors: EINVAL (unknown ticket), ESTATE (not done), or the request's own failure code. */
int nmfa_server_result(nmfa_server *s, uint64_t ticket, double *E, int64_t *E_int, int8_t *spins,
                       double *latency_ms);

/* Forget a finished request and free its host-side results. Errors: EINVAL, ESTATE (not finished). */
int nmfa_server_release(nmfa_server *s, uint64_t ticket);

/* Cancel a request: a queued one is dropped at once, a running one at the next round boundary.
 * Errors: EINVAL (unknown ticket), ESTATE (already finished). */
int nmfa_server_cancel(nmfa_server *s, uint64_t ticket);

/* Counters of the server. Errors: EINVAL. */
int nmfa_server_stats_get(nmfa_server *s, nmfa_server_stats *out);

/* Cancel whatever is queued, let running requests stop at the next round, join the scheduler
 * and free everything (NULL is ignored). */
void nmfa_server_destroy(nmfa_server *s);

#ifdef __cplusplus
}
#endif

#endif /* NMFA_H */
