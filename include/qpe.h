/*
 * qpe.h -- C ABI of the MI355X (gfx950) QPE statevector emulator.
 *
 * Operation (paper section 2, Fig. 1, the QPE circuit): for a target matrix
 * U (d x d, d = 2^N_mat), an input state psi (d) and N_meas measurement
 * qubits (N = 2^N_meas), return the measurement probabilities
 *
 *     A[m, :] = 2^-N_meas * sum_{j<N} exp(-2 pi i j m / N) U^j psi
 *     P(m)    = sum_r |A[m, r]|^2,         m = 0 .. N-1.
 *
 * The circuit: H on every measurement qubit of |0..0>, then for k = 0..n-1
 * the qubit carrying bit k of the register integer controls U^(2^k), then the
 * inverse QFT on the measurement register, then measurement. The readout is
 * the "norm of the final statevector" of the paper (section 3) marginalised
 * over the target register. Bit k of the outcome m is the qubit that
 * controlled U^(2^k); the peak of an eigenvector input with eigenphase phi
 * lies at m ~ phi * N.
 *
 * Conventions common to every entry point:
 *  - complex128 = two doubles (re, im), complex64 = two floats (re, im);
 *    matrices are row-major: (U v)_r = sum_c U[r*d + c] v_c.
 *  - Every data pointer is a DEVICE pointer owned by the caller; the library
 *    never allocates or frees device memory. Scratch memory comes from the
 *    caller's workspace (size from qpe_workspace_size), 256-byte aligned.
 *  - Work is enqueued asynchronously on the context's HIP stream; results are
 *    valid after the caller synchronises that stream. A call returns before
 *    the device work is done, so device faults surface as QPE_ERR_HIP from a
 *    later call.
 *  - Argument, size and alignment checks run on the host before any HIP call
 *    and need no device. No function aborts and no C++ exception crosses the
 *    ABI. On error nothing has been enqueued.
 *  - Not thread-safe per context; distinct contexts are independent.
 */
#ifndef QPE_H
#define QPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum qpe_status {
  QPE_OK = 0,
  QPE_ERR_ARG = 1,         /* null pointer, unknown form/flag, bad count   */
  QPE_ERR_SIZE = 2,        /* N_meas / N_mat (or a GEMM size) out of range */
  QPE_ERR_ALIGN = 3,       /* a device pointer is not 16-byte aligned       */
  QPE_ERR_WORKSPACE = 4,   /* workspace null, too small or not 256-aligned */
  QPE_ERR_OOM = 5,         /* host allocation for the context failed       */
  QPE_ERR_NO_DEVICE = 6,   /* no HIP device, or the device index is invalid*/
  QPE_ERR_HIP = 7,         /* a HIP runtime call or a kernel launch failed */
  QPE_ERR_UNSUPPORTED = 8  /* valid request the library does not implement */
} qpe_status;

/* Arithmetic form of the statevector path.
 *  QPE_FORM_FP64 : complex128 state; FP64 matrix-core GEMMs throughout.
 *  QPE_FORM_MIXED: complex64 state; the controlled products run on the
 *                  matrix cores as split products accumulated in FP32: the
 *                  state (scaled by a power of two) and the operator
 *                  (scaled by 2^14) as two FP16 pieces each, three partial
 *                  products (QPE_SPLIT_BF16, and runs without the polar
 *                  step: three BF16 pieces each, six partial products);
 *                  the inverse QFT runs in FP32 and the readout sums in
 *                  FP64; the target register is rotated first
 *                  (QPE_MIX_TARGET).
 * In both forms the powers U^(2^k) are formed in FP64. */
typedef enum qpe_form { QPE_FORM_FP64 = 0, QPE_FORM_MIXED = 1 } qpe_form;

/* Run flags. */
enum {
  /* Skip the Newton-Schulz re-unitarisation of the powers. Required when U
   * is not unitary (the paper's analytic test problem, section 3, builds
   * U = P Lambda P^-1 with a non-unitary P). */
  QPE_NO_POLAR = 1u << 0,
  /* Prefix-doubling form of the controlled stage. The measurement register
   * starts in |0...0> (Fig. 1), so after the H layer and the controlled
   * steps for bits below k, rows [2^k, 2^(k+1)) of the state equal rows
   * [0, 2^k) times V_k^T. With this flag step k computes exactly those rows
   * from rows [0, 2^k): 2^n - 1 row products instead of n 2^(n-1), each row
   * receiving the same sequence of products as in the gate route. Same P. */
  QPE_PREFIX_DOUBLING = 1u << 1,
  /* Target rotation (on by default in QPE_FORM_MIXED for n_mat >= 5 unless
   * QPE_NO_POLAR is set). Before the run U <- M U M^H and psi <- M psi with
   * M = D2 H D1 / sqrt(d): H the Walsh-Hadamard matrix, D1 a diagonal of
   * signs and D2 one of unit phases, both derived from a hash of the bits of
   * U and psi (of four candidate sign diagonals, the one that leaves the
   * smallest peak weight max_i |(M psi)_i|^2 / ||psi||^2). M is unitary, so
   * P(m), a marginal over the target register (section 2, Fig. 1), is
   * unchanged in exact arithmetic. Why: the mixed form's matrix-core
   * products round each 16-term sum with an error of up to a few ulp; for
   * state rows spread over the d components these errors average out, for
   * rows concentrated on a few basis vectors (e.g. an eigenvector close to
   * a basis vector) they add up coherently over the n steps (up to 1.9e-6
   * of total probability at N_meas = 16 to 20 without it). M spreads such
   * inputs. Cost: a few Walsh-Hadamard passes over U (FP64, no d x d
   * products). Not a default with QPE_NO_POLAR: for a non-unitary U the
   * rotated products cancel more (measured on the paper's analytic problem:
   * errors up to 2.6e-5 rotated against 1.2e-6 unrotated at d = 1024).
   * qpe_run_state rotates the final statevector back. QPE_MIX_TARGET forces
   * the rotation on (any form, n_mat >= 1); QPE_NO_MIX_TARGET turns it off;
   * both: QPE_ERR_ARG. */
  QPE_MIX_TARGET = 1u << 2,
  QPE_NO_MIX_TARGET = 1u << 3,
  /* QPE_FORM_MIXED: run the controlled products as split-BF16 products
   * (three BF16 pieces per operand, six piece products) instead of the
   * default split-FP16 ones (two FP16 pieces per operand, three piece
   * products: half the matrix-core work). Without the polar step
   * (QPE_NO_POLAR) the split-BF16 scheme always runs: the FP16 pieces are
   * scaled for the row norms a unitary U keeps, and a non-unitary U can
   * grow them past the FP16 range. */
  QPE_SPLIT_BF16 = 1u << 4
};

/* Report flags (qpe_report.flags). */
enum {
  QPE_REPORT_NOT_UNITARY = 1u << 0, /* max|V^H V - I| above 1e-6 at some step */
  QPE_REPORT_NUMERIC = 1u << 1,     /* NaN/Inf in P, or |sum P - |psi|^2| > 1e-4*|psi|^2 */
  /* mixed form, n_mat >= 5: the input the matrix cores see (M psi when
   * rotated, else psi) holds more than half of its norm on one basis vector
   * (input_peak > 0.5), the case whose rounding errors add up coherently */
  QPE_REPORT_CONCENTRATED = 1u << 2
};

/* Limits. d = 2^n_mat, N = 2^n_meas. */
#define QPE_MAX_N_MEAS 30
#define QPE_MAX_N_MAT 15
#define QPE_MAX_TOTAL_QUBITS 34 /* n_meas + n_mat */

/* One QPE instance. U: device complex128 [d*d]; psi: device complex128 [d]
 * (not renormalised: sum_m P(m) = ||psi||^2 up to rounding); prob: device
 * float64 [N], written. U and psi are read only. */
typedef struct qpe_problem {
  int32_t n_meas; /* 1 .. QPE_MAX_N_MEAS                       */
  int32_t n_mat;  /* 0 .. QPE_MAX_N_MAT                        */
  const void *U;
  const void *psi;
  double *prob;
} qpe_problem;

/* Device-written diagnostics, one per instance (caller-owned device memory,
 * 8-byte aligned). unitarity_defect is the largest max-norm of V^H V - I met
 * before each Newton-Schulz step (the powers k = 3, 7, 11, ... and the last
 * one, k = n_meas - 1; 0 when QPE_NO_POLAR); prob_sum = sum_m P(m);
 * psi_norm2 = ||psi||^2; input_peak = max_i |x_i|^2 / ||psi||^2 for the input
 * x of the state path (M psi when the target register was rotated, else
 * psi). */
typedef struct qpe_report {
  double unitarity_defect;
  double prob_sum;
  double psi_norm2;
  double input_peak;
  uint32_t flags;
  uint32_t reserved;
} qpe_report;

typedef struct qpe_ctx qpe_ctx;

/* Create a context bound to HIP device `device` and HIP stream `stream`
 * (a hipStream_t; NULL = the legacy default stream). Host memory only.
 * For tests of the error path: if the environment variable QPE_FAULT_INJECT
 * holds a number N >= 1 when the context is created, the N-th checked HIP
 * call made for it is not made and is reported as failed (QPE_ERR_HIP,
 * qpe_last_error says so); later calls run normally.
 * Errors: QPE_ERR_ARG (ctx NULL), QPE_ERR_NO_DEVICE, QPE_ERR_OOM. */
qpe_status qpe_ctx_create(qpe_ctx **ctx, int device, void *stream);

/* Rebind the context to another stream on the same device. */
qpe_status qpe_ctx_set_stream(qpe_ctx *ctx, void *stream);

/* Destroy a context (host memory only; does not synchronise). NULL is OK. */
qpe_status qpe_ctx_destroy(qpe_ctx *ctx);

/* Workspace bytes qpe_run needs for these problems, form and flags. Only the
 * size fields of the problems are read (pointers may be NULL). Host only.
 * Errors: QPE_ERR_ARG, QPE_ERR_SIZE. */
qpe_status qpe_workspace_size(const qpe_problem *problems, int count, int form,
                              unsigned flags, size_t *bytes);

/* Run `count` independent QPE instances (paper section 2, Fig. 1) and write
 * each instance's probability vector. problems: HOST array of `count`
 * entries. workspace: device, >= qpe_workspace_size bytes, 256-aligned; its
 * contents on entry are ignored. report: device array of `count` qpe_report,
 * or NULL. count > 1 runs the instances batched (uneven sizes allowed).
 * Nothing is allocated; the call is asynchronous on the context stream and
 * may be captured in a HIP graph.
 * Errors: QPE_ERR_ARG, QPE_ERR_SIZE, QPE_ERR_ALIGN, QPE_ERR_WORKSPACE,
 * QPE_ERR_HIP. */
qpe_status qpe_run(qpe_ctx *ctx, const qpe_problem *problems, int count, int form,
                   unsigned flags, void *workspace, size_t workspace_bytes,
                   qpe_report *report);

/* One instance as qpe_run (count 1), also returning the final statevector:
 * the paper's emulator outputs the statevector after the inverse QFT
 * (section 3), whose norms give the outcome distribution. state_out
 * (device, caller-owned, N*d elements) receives A[m, r] of the formula at the
 * top of this header, row-major in natural outcome order m: complex64 for
 * QPE_FORM_MIXED, complex128 for QPE_FORM_FP64 (a run with the target
 * rotation rotates it back). prob and report are written as by qpe_run.
 * Same workspace as qpe_run for this one problem.
 * Errors: as qpe_run; QPE_ERR_ALIGN if state_out is not aligned to its
 * element size. */
qpe_status qpe_run_state(qpe_ctx *ctx, const qpe_problem *problem, int form, unsigned flags,
                         void *workspace, size_t workspace_bytes, void *state_out,
                         qpe_report *report);

/* qpe_run without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). It calls no hipMalloc/hipFree and no
 * allocating library routine: the workspace is a static device array of
 * QPE_STATIC_WORKSPACE_BYTES that each device the library runs on holds from
 * the first qpe_ctx_create on that device until the process ends. Every call
 * on one device shares that array and keeps the last call's contents (a run
 * ignores them on entry), so calls that overlap in time on one device (other
 * streams, other contexts, other host threads) race and give wrong results:
 * serialise them. Arguments, outputs and errors as qpe_run; problems whose
 * qpe_workspace_size exceeds QPE_STATIC_WORKSPACE_BYTES: QPE_ERR_WORKSPACE
 * (qpe_last_error gives both sizes), nothing enqueued; the array's address
 * unavailable on the device: QPE_ERR_HIP. */
#define QPE_STATIC_WORKSPACE_BYTES (64u << 20)
qpe_status qpe_run_static(qpe_ctx *ctx, const qpe_problem *problems, int count, int form,
                          unsigned flags, qpe_report *report);

/* Host-only pre-flight: the status qpe_run would return for these arguments
 * before it touches the context or the device (QPE_OK if they are valid).
 * Never dereferences device pointers. */
qpe_status qpe_check_run(const qpe_problem *problems, int count, int form, unsigned flags,
                         const void *workspace, size_t workspace_bytes, const void *report);

/* ---- stage entry points (one step of the path each, for per-step checks) ---- */

/* Powers of U (the controlled operators of Fig. 1): V_k = U^(2^k) for
 * k = 0 .. count_k-1, by FP64 repeated squaring; the squares of k = 3, 7,
 * 11, ... and of the last k (count_k - 1) are followed by one Newton-Schulz
 * step X <- X (3I - X^H X)/2 unless QPE_NO_POLAR (a squaring doubles the
 * unitarity defect, one step takes a defect delta to about 1.5 delta^2, so
 * correcting every fourth power keeps it within about eight times the
 * rounding level; qpe_run uses the same schedule with count_k = n_meas).
 * U: device complex128 [d*d]; V_out: device complex128 [count_k][d][d];
 * workspace: >= qpe_powers_workspace_size bytes; report: device qpe_report
 * or NULL (only unitarity_defect is written). 1 <= count_k <= 30. */
qpe_status qpe_powers_workspace_size(int n_mat, size_t *bytes);
qpe_status qpe_powers(qpe_ctx *ctx, int n_mat, const void *U, int count_k,
                      unsigned flags, void *V_out, void *workspace,
                      size_t workspace_bytes, qpe_report *report);

/* One controlled step of Fig. 1 on a caller-held state: for every row j of
 * state (N x d, row-major) whose bit k is set, state[j,:] <- state[j,:] V^T
 * (i.e. the target vector s becomes V s). V: device complex128 [d*d]. state:
 * complex128 (QPE_FORM_FP64) or complex64 (QPE_FORM_MIXED), updated in place.
 * Uses the same operator preparation and GEMM kernels as qpe_run.
 * 0 <= k < n_meas. workspace >= qpe_controlled_step_workspace_size. */
qpe_status qpe_controlled_step_workspace_size(int n_meas, int n_mat, int form, size_t *bytes);
qpe_status qpe_controlled_step(qpe_ctx *ctx, int n_meas, int n_mat, int form, int k,
                               const void *V, void *state, void *workspace,
                               size_t workspace_bytes);

/* Inverse QFT on the measurement register followed by the readout (the last
 * two stages of Fig. 1): state (N x d, complex128 for FP64, complex64 for
 * MIXED) is transformed in place into a digit-reversed row order (contents
 * unspecified afterwards) and prob[m] = sum_r |A[m, r]|^2 is written
 * (device float64 [N]). workspace >= qpe_iqft_workspace_size: the twiddle
 * tables and, for n_meas >= 12 except 17 (where the readout is summed
 * inside the last DFT pass, from per-row partial sums over column groups),
 * those partial sums. qpe_run and qpe_run_state take the same passes and
 * sums, so all three return the same prob bit for bit. */
qpe_status qpe_iqft_workspace_size(int n_meas, int n_mat, int form, size_t *bytes);
qpe_status qpe_iqft_probs(qpe_ctx *ctx, int n_meas, int n_mat, int form, void *state,
                          double *prob, void *workspace, size_t workspace_bytes);

/* ---- phase estimators (paper section 4.2, precision evaluation) ----
 * From each problem's probability vector P = problems[i].prob (device
 * float64 [N], N = 2^n_meas, as written by qpe_run; only n_meas and prob are
 * read), out[i] receives
 *   argmax_index   : the m with the largest P(m), the smallest such m on a
 *                    tie; NaN entries are never chosen (-1 if all are NaN);
 *   argmax_phase   : argmax_index / N, the max-norm estimator (NaN if -1);
 *   weighted_phase : sum_m P(m) (m / N) / sum_m P(m), the weighted-average
 *                    estimator as the paper states it (biased for phases
 *                    near the 0/1 wrap);
 *   circular_phase : arg(sum_m P(m) exp(2 pi i m / N)) / (2 pi) in [0, 1),
 *                    the circular mean (no bias at the wrap);
 *   prob_sum       : sum_m P(m).
 * Sums run in FP64 over a partition of m that depends only on N, so the
 * results are reproducible. problems: HOST array; out: DEVICE array of
 * `count` qpe_estimates, 8-byte aligned; workspace: device, 256-aligned,
 * >= qpe_estimate_workspace_size(count). Asynchronous on the context stream.
 * Errors: QPE_ERR_ARG, QPE_ERR_SIZE, QPE_ERR_ALIGN, QPE_ERR_WORKSPACE,
 * QPE_ERR_HIP. */
typedef struct qpe_estimates {
  double argmax_phase;
  double weighted_phase;
  double circular_phase;
  double prob_sum;
  int64_t argmax_index;
  int64_t reserved;
} qpe_estimates;
qpe_status qpe_estimate_workspace_size(int count, size_t *bytes);
qpe_status qpe_estimate(qpe_ctx *ctx, const qpe_problem *problems, int count,
                        qpe_estimates *out, void *workspace, size_t workspace_bytes);

/* Complex FP64 GEMM on the matrix cores (the building block of the powers):
 * C = alpha * op(A) * op(B) + beta * Cin, op in {'N','T','C'} (none,
 * transpose, conjugate transpose); op(A) is M x K, op(B) is K x N; all
 * complex128 row-major with leading dimensions lda/ldb/ldc in elements.
 * alpha/beta: complex (re, im) pairs. Cin may equal C (then read before
 * write per element) or be NULL when beta == 0. 1 <= M, N, K <= 65536. */
qpe_status qpe_zgemm(qpe_ctx *ctx, char opA, char opB, int M, int N, int K,
                     const double *alpha, const void *A, int lda, const void *B, int ldb,
                     const double *beta, const void *Cin, int ldcin, void *C, int ldc);

/* ---- per-kernel timing (HIP events on the context stream) ----
 * When enabled, every launch of the kernel classes below is bracketed by a
 * pair of HIP events recorded on the context stream (a pool of `max_pairs`
 * pairs is created on the host by the enable call; launches beyond the pool
 * go untimed). qpe_ctx_read_timing synchronises the recorded events and
 * returns the number of timed launches of a class and their summed
 * duration. Resetting frees the pool for reuse. Not capturable. */
enum {
  QPE_TIMER_CTRL_GEMM = 0, /* controlled-step kernels (all forms)          */
  QPE_TIMER_POWERS = 1,    /* FP64 squaring and Newton-Schulz kernels       */
  QPE_TIMER_SPLIT = 2,     /* separate operator-split passes (a split made
                              in the square's epilogue or the Newton-Schulz
                              update is timed with the power chain)        */
  QPE_TIMER_QFT = 3,       /* inverse-DFT passes                           */
  QPE_TIMER_PROB = 4,      /* readout                                      */
  QPE_TIMER_HLAYER = 5,    /* Hadamard layer                               */
  QPE_TIMER_COUNT = 6
};
qpe_status qpe_ctx_enable_timing(qpe_ctx *ctx, int max_pairs);
/* Timer classes that record events: bit c set = class c timed (all by
 * default); launches of the other classes are not bracketed, so their
 * events cost nothing. QPE_ERR_ARG for NULL ctx or bits beyond
 * QPE_TIMER_COUNT. */
qpe_status qpe_ctx_set_timing_mask(qpe_ctx *ctx, unsigned mask);
qpe_status qpe_ctx_reset_timing(qpe_ctx *ctx);
qpe_status qpe_ctx_read_timing(qpe_ctx *ctx, int timer, int *launches, double *total_ms);

/* ---- kernel variants (tile shapes), chosen by the autotuner below ----
 * Each kernel class has variants 1..count (different tile shapes and
 * pipelining); 0 selects the built-in default. A context applies its
 * choice to every later call. All variants compute the same result up to
 * rounding order. */
enum {
  QPE_KERNEL_CTRL_MIXED = 0, /* split-FP16 / split-BF16 controlled GEMM
                                (d >= 32); variants 8 (128 x 256 tiles)
                                and 9 (the same, one persistent workgroup
                                per CU; the default for d >= 256) exist
                                for split FP16 only                   */
  QPE_KERNEL_ZGEMM = 1,      /* FP64 GEMM of the power chain (the
                                Gram products of n_mat = 10 and 11 run
                                a fixed stream-K plan instead)        */
  QPE_KERNEL_CTRL_F64 = 2,   /* FP64 controlled GEMM (d >= 32)        */
  /* Batched runs (count > 1). One setting per context: n_mat is checked
   * but the choice applies to every instance size. */
  QPE_KERNEL_BATCH_CTRL = 3, /* grouped controlled step, d >= 128: 1 in-step
                                schedule (d = 128), 2 (default) ping-pong with
                                one tile per workgroup, 3 ping-pong with the
                                split-FP16 step of the d >= 256 instances on
                                one persistent workgroup per CU (when those
                                instances share one d) */
  QPE_KERNEL_BATCH_GEMM = 4, /* grouped FP64 power-chain products: 1 32x32
                                tiles (default), 2 64x64 tiles for d >= 64 */
  QPE_KERNEL_BATCH_SCHED = 5, /* schedule of a batched run with the polar
                                 step, and of a single run's prefix-doubling
                                 form: 1 one stream, 2 (default) the power
                                 chain on a second stream of the context
                                 (created with its events by qpe_ctx_create;
                                 if that failed, by the first such run), so
                                 that the power products of step k+1 overlap
                                 the controlled products of step k; joined
                                 back into the context stream before the run
                                 returns, also when it fails. While the
                                 power-chain timer class records (timing
                                 enabled and QPE_TIMER_POWERS in the mask:
                                 its events go to the context stream), or in
                                 qpe_run_static (which creates nothing), one
                                 stream. The setting of n_mat 0 applies. */
  QPE_KERNEL_COUNT = 6
};
qpe_status qpe_kernel_variants(int kernel_class, int *count);
/* n_mat selects the operator size the choice applies to (0..QPE_MAX_N_MAT),
 * or -1 for every size. */
qpe_status qpe_ctx_set_variant(qpe_ctx *ctx, int kernel_class, int n_mat, int variant);

/* The variant the context currently uses for a class and operator size. */
qpe_status qpe_ctx_get_variant(const qpe_ctx *ctx, int kernel_class, int n_mat, int *variant);

/* Autotuner (the tile shapes of the batched-GEMM pattern are picked by
 * measurement, not fixed): for each kernel class this problem uses (the
 * power-chain GEMM; the controlled GEMM of its form when d >= 32), run the
 * whole circuit with every variant of that class, 0 (the built-in default)
 * included, and keep the fastest for the problem's n_mat in the context. The
 * timed runs are one warm-up plus `reps` (1..1000) circuits per variant,
 * bracketed by HIP events on the context stream; the call SYNCHRONISES that
 * stream and is not capturable. The problem's prob vector is overwritten.
 * chosen: host int[QPE_KERNEL_COUNT], the variant in place for every class
 * afterwards (unchanged for classes not tuned). class_ms: host
 * double[QPE_KERNEL_COUNT * QPE_TUNE_MAX_VARIANTS] or NULL: mean ms per
 * circuit of each (class, variant) tried, -1 where not tried.
 * Errors: as qpe_run; QPE_ERR_ARG for reps out of range or chosen NULL. */
#define QPE_TUNE_MAX_VARIANTS 12
qpe_status qpe_autotune(qpe_ctx *ctx, const qpe_problem *problem, int form, unsigned flags,
                        void *workspace, size_t workspace_bytes, int reps, int *chosen,
                        double *class_ms);

/* The same for a batched run (the grouped kernels of `count` >= 2 problems):
 * each batched class this batch uses (QPE_KERNEL_BATCH_GEMM and, with the
 * polar step, QPE_KERNEL_BATCH_SCHED when any instance has n_meas >= 2,
 * QPE_KERNEL_BATCH_CTRL in the mixed form when any instance has
 * n_mat >= 7) is timed over whole batched runs, every
 * variant in turn, and the fastest is kept. Arguments, outputs and errors
 * as qpe_autotune, with the problems, count and workspace of qpe_run;
 * every problem's prob vector is overwritten. */
qpe_status qpe_autotune_batch(qpe_ctx *ctx, const qpe_problem *problems, int count, int form,
                              unsigned flags, void *workspace, size_t workspace_bytes, int reps,
                              int *chosen, double *class_ms);

/* ---- misc ---- */

/* Static text for a status code (never NULL). */
const char *qpe_status_string(int status);

/* Text of the most recent error on this context (HIP error name included),
 * or "" if none. Valid until the next call on ctx. */
const char *qpe_last_error(const qpe_ctx *ctx);

/* Library version, "major.minor.patch". */
const char *qpe_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QPE_H */
