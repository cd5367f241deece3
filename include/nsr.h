/*
 * nsr.h -- C ABI of a high-order Newton-Schulz / Richardson solver for SPD
 * systems on AMD Instinct MI355X (gfx950).
 *
 * Method: Stotsky, "Convergence Rate Improvement of Richardson and
 * Newton-Schulz Iterations" (arXiv 2008.11480).
 *   problem            A theta* = b, A symmetric positive definite   (eq. ae1)
 *   preconditioner     S^{-1} = I / alpha                            (Section 2)
 *   Newton-Schulz      G_k = G_{k-1} P(F_{k-1}),  F = I - A G,
 *                      P(F) = I + F + ... + F^{n-1}                  (eqs. ns, fk1)
 *   factorized forms   (I+F)(I+F^2)(I+F^4)..., Horner, unified (p,w) (Section 4,
 *                                                                     Appendix)
 *   composite form     double Newton-Schulz                          (Section 5.1)
 *   Richardson         theta_k = theta_{k-1} + G_k (b - A theta_{k-1}) (eq. redttk1)
 *
 * The residual is kept on the right, F = I - A G and G <- G P(F); every
 * iterate is a polynomial in A, so this is the paper's left-residual
 * iteration with the products mirrored, and F_{k+1} = F_k^n holds exactly.
 *
 * Conventions
 *   - Every call returns an int status: NS_OK (0) or a negative ns_status.
 *     ns_status_string() names a status, ns_last_error() gives the message of
 *     the calling thread's most recent failure.  No C++ exception and no
 *     abort() crosses this boundary.
 *   - Matrices are row-major float64 with a leading dimension (ld >= n).
 *     All matrix and vector pointers are DEVICE pointers unless stated.
 *     The iterates G, F live in the workspace in the solver's precision
 *     (float64, or float32 with bf16 copies); A, b, theta and the Richardson
 *     residual are always float64.
 *   - The caller owns A, b, theta and the workspace; the library never calls
 *     hipMalloc on the solve path.  A is borrowed from ns_bind() until the
 *     next ns_bind() or ns_destroy(); it is never written.
 *   - All work is enqueued on the stream given to ns_create() (a hipStream_t
 *     passed as void*; NULL is the default stream).  Calls that return a
 *     host-visible number (alpha_out, fnorm_out, reports) synchronize that
 *     stream before returning.
 *   - A solver handle is not thread-safe: one handle per host thread.
 */
#ifndef NSR_H
#define NSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NS_OK = 0,
  NS_EINVAL = -1,      /* bad argument, unsupported option combination      */
  NS_ENOTSPD = -2,     /* alpha <= 0 or non-finite: A cannot be SPD          */
  NS_EDIVERGED = -3,   /* ||F_k||_F grew above ||F_0||_F or became non-finite */
  NS_ENOCONV = -4,     /* resid_tol not reached within k_max / refine_max    */
  NS_ENOMEM = -5,      /* workspace too small                                */
  NS_EHIP = -6,        /* a HIP runtime call failed                          */
  NS_EBUSY = -7,       /* batch ticket not finished (ns_batch_poll, wait=0)  */
  NS_EPRECISION = -8,  /* precision mode cannot reach the tolerance          */
  NS_ESTATE = -9       /* call out of order (e.g. ns_step before ns_init_scale) */
} ns_status;

typedef enum {
  NS_PREC_FP64 = 0,       /* every product and vector in float64             */
  NS_PREC_FP32 = 1,       /* products in float32 MFMA, Richardson in float64 */
  NS_PREC_MIXED_BF16 = 2, /* powers of F in bf16 MFMA (fp32 accumulate), the
                             residual and G-side products in float32,
                             Richardson in float64                           */
  NS_PREC_MIXED_SPLIT = 3 /* as NS_PREC_MIXED_BF16, but the residual, G-side
                             and merge products are float32-class products
                             of split half-precision operands on the
                             half-precision matrix cores (ns_gemm_f32_split:
                             22-bit operands, float32 accumulation)          */
} ns_precision;

typedef enum {
  NS_SCALE_FROBENIUS = 0, /* alpha = ||A||_F  (lambda_max <= ||A||_F, so the
                             splitting condition 2S - A > 0 holds)           */
  NS_SCALE_INF_HALF = 1,  /* alpha = ||A||_inf / 2 + eps (Section 2)         */
  NS_SCALE_DIAG = 2       /* S = diag(A) (Section 2, SDD matrices; converges
                             when 2S - A is positive definite).  F = I - A S^-1
                             is then not symmetric: every product runs in full.
                             Float64 and float32 modes.                       */
} ns_scale;

typedef enum {
  NS_FACT_HORNER = 0,        /* Horner's scheme, eq. (z1): n mmm per step      */
  NS_FACT_SQUARING = 1,      /* (I+F)(I+F^2)(I+F^4)..., n = 2^s: 2s mmm
                                (Tables 1-2, orders 2, 4, 8)                   */
  NS_FACT_TABLE = 2,         /* nested programs: order 11 (Table 2, second
                                form, 6 mmm), 15 (Table 3, 7 mmm), 45
                                (eqs. ex1-ex3, 10 mmm); mmm counts include the
                                step's residual                                */
  NS_FACT_UNIFIED = 3,       /* eqs. (xa2)-(zi1), n = w(p+1): p+w+1 mmm        */
  NS_FACT_UNIFIED_PLUS1 = 4, /* eq. (ztab2), n = w(p+1)+1                      */
  NS_FACT_COMPOSITE_DOUBLE = 5, /* double Newton-Schulz, Section 5.1; inner
                                  sums by squaring (n = 2^s), else Horner     */
  NS_FACT_SRI = 6,           /* the two-loop algorithm of Remark 2 ([sri]):
                                Z_k = Z_{k-1} P_p(I - A Z_{k-1}),
                                G_k = G_{k-1} + Z_k F_{k-1} (mirrored); for
                                comparison                                     */
  NS_FACT_COMPOSITE_GENERAL = 7 /* composite expansion of eqs. (gkgen1)-(ga1):
                                w parallel power series of rates x_i = m_i^k
                                (ns_set_composite_rates) and an order-n NS
                                loop, n >= 1: F_k = F_{k-1}^n Gamma_c          */
} ns_factorization;

/* Why a phase of richardson_ns_solve ended (ns_solve_report.*_stop). */
typedef enum {
  NS_STOP_NONE = 0,
  NS_STOP_F_TOL = 1,        /* ||F_k||_F <= f_tol                              */
  NS_STOP_FLOOR = 2,        /* rounding floor, found by either of two tests.
                               Error law: ||F_{k-1}|| < 1 and ||F_k|| >
                               1e3 ||F_{k-1}||^n (eq. fk1 bounds ||F_k|| by
                               ||F_{k-1}||^n in exact arithmetic; the double
                               Newton-Schulz exponent grows at least n-fold
                               per step).  Ratio: ||F_k|| > ||F_{k-1}|| / 2
                               while ||F_k^2|| <= ||F_k|| / 4, which exact
                               iterates cannot show (F_k = F_{k-1}^n).  Not
                               used by the general composite and [sri] forms
                               (ratio test only)                              */
  NS_STOP_K_MAX = 3,
  NS_STOP_DIVERGED = 4,     /* ||F_k|| > ||F_0|| or non-finite                 */
  NS_STOP_RESID_TOL = 5,    /* ||b - A theta|| / ||b|| <= resid_tol            */
  NS_STOP_REFINE_MAX = 6,
  NS_STOP_REFINE_STALL = 7, /* less than a factor 2 over 3 refinement steps    */
  NS_STOP_PRECISION = 8     /* batched float32 attempt: ||F_k||_F >= 1/2 and not
                               halving after the steps that resolve every
                               eigenvalue float32 can represent; re-solved in
                               float64                                        */
} ns_stop_reason;

typedef struct ns_solver ns_solver;

/* Bytes of device workspace a solver of dimension n needs for the given
 * precision.  composite = 0: the classical and table forms; 1: also the
 * double Newton-Schulz loop (Section 5.1), the [sri] form and the general
 * composite with one loop; 2 or 3: the general composite with that many
 * loops.  ns_create takes the largest level the given bytes cover.  Returns
 * 0 for n < 1, an unknown precision or composite outside 0..3. */
size_t ns_workspace_bytes(int64_t n, int precision, int composite);

/* Create a solver for n x n systems on HIP device `device`, enqueuing on
 * `hip_stream`.  `workspace` is a device buffer of `bytes` bytes (at least
 * ns_workspace_bytes(n, precision, composite) with composite = 1 if the
 * composite form will be used, 256-byte aligned), owned by the caller and
 * used exclusively by this solver until ns_destroy().  Errors: NS_EINVAL (n<1,
 * unknown precision, NULL out/workspace, misaligned workspace), NS_ENOMEM
 * (bytes too small), NS_EHIP. */
int ns_create(int device, void* hip_stream, int64_t n, int precision,
              void* workspace, size_t bytes, ns_solver** out);

int ns_destroy(ns_solver* s);

/* Borrow A (device, row-major float64, lda >= n, symmetric positive definite;
 * symmetry is assumed, not checked).  Resets the iteration state.  In the
 * float32 / mixed modes this also enqueues a float32 copy of A into the
 * workspace (used by the residual products I - A G).  Errors: NS_EINVAL
 * (NULL, lda < n), NS_EHIP. */
int ns_bind(ns_solver* s, const double* A, int64_t lda);

/* Section 2 (preconditioner S): compute alpha (NS_SCALE_FROBENIUS: ||A||_F;
 * NS_SCALE_INF_HALF: max row sum / 2 + eps) and S = alpha I, or
 * (NS_SCALE_DIAG) S = diag(A), reporting alpha = max_i A_ii; set G_0 = S^-1
 * (kept implicit, never materialised) and F_0 = I - A G_0, and return alpha
 * and ||F_0||_F (either out pointer may be NULL).  Errors: NS_ESTATE (no A
 * bound), NS_ENOTSPD (alpha, or a diagonal entry, not finite or <= 0),
 * NS_EINVAL (unknown scale; NS_SCALE_DIAG in the mixed mode, whose bf16
 * products assume symmetric powers of F). */
int ns_init_scale(ns_solver* s, int scale, double eps, double* alpha_out,
                  double* fnorm0_out);

/* One Newton-Schulz step of order `order` evaluated by `factorization`
 * (p, w used by the unified forms only): G_k = G_{k-1} P(F_{k-1}), then
 * F_k = I - A G_k, eq. (ns) and (fk1).  For NS_FACT_COMPOSITE_DOUBLE it is
 * one step of eqs. (gamk11)-(fks1) (the first call also forms L_0).  Writes
 * ||F_k||_F to fnorm_out when non-NULL (this synchronizes the stream).
 * Errors: NS_ESTATE (before ns_init_scale), NS_EINVAL (order < 2, order not
 * matching the factorization, factorization unsupported for the precision). */
int ns_step(ns_solver* s, int order, int factorization, int p, int w,
            double* fnorm_out);

/* Symmetric power products (default on).  The products among powers of F
 * (F^2, F^4, the identity-offset assembly; Tables 1-2) are polynomials in F
 * and symmetric in exact arithmetic; with this on, each is computed on the
 * tiles on or above the diagonal and mirrored (n^2 (n + 1) flop instead of
 * 2 n^3).  The residual I - A G and the G-side / merge products always run in
 * full: Newton-Schulz corrects a perturbation of G only when F is the exact
 * residual of the G it multiplies.  Float64 mode only. */
int ns_set_symmetric(ns_solver* s, int enable);

/* Loops of NS_FACT_COMPOSITE_GENERAL: w in 1..3 power series with orders
 * rates[i] in 1..64 (x_i = rates[i]^k after k steps; a rate of 1 keeps
 * T_i = S^-1).  Needs a workspace of ns_workspace_bytes(n, precision,
 * w) or more; set before the first composite step after ns_init_scale.
 * Orders 2^s use the squaring sums, others Horner.
 * Errors: NS_EINVAL, NS_ESTATE. */
int ns_set_composite_rates(ns_solver* s, int w, const int* rates);

/* Copy the current G_k into G_out (device, row-major float64, ldg >= n;
 * converted from float32 in the float32 / mixed modes). */
int ns_get_G(ns_solver* s, double* G_out, int64_t ldg);

/* Copy the current F_k = I - A G_k into F_out (device, float64, ldf >= n). */
int ns_get_F(ns_solver* s, double* F_out, int64_t ldf);

/* One Richardson step with the current G: r = b - A theta (float64),
 * theta += G r (eq. redttk1 with omega = G).  b, theta: device float64 of
 * length n.  Writes ||r||_2 (of the residual BEFORE the update) to
 * rnorm_out when non-NULL. */
int ns_richardson_step(ns_solver* s, const double* b, double* theta, double* rnorm_out);

typedef struct {
  int order;          /* n >= 2                                              */
  int factorization;  /* ns_factorization                                    */
  int p, w;           /* unified-form parameters                             */
  int k_max;          /* at most this many Newton-Schulz steps (<= 64)       */
  int refine_max;     /* at most this many refinement-only Richardson steps  */
  int floor_detect;   /* 1: stop Newton-Schulz at the rounding floor         */
  int scale;          /* ns_scale                                            */
  double eps;         /* for NS_SCALE_INF_HALF                               */
  double f_tol;       /* stop Newton-Schulz when ||F_k||_F <= f_tol          */
  double resid_tol;   /* target of ||b - A theta||_2 / ||b||_2               */
  int theta0_mode;    /* 0: theta_0 = G_0 b;  1: theta_0 = 0;  2: caller's   */
  int accel_q;        /* 0: Richardson with omega_k = G_k (eq. redttk1).
                         q >= 1 (composite form only): the high-order
                         accelerator of eq. (ttk1), omega_k = L_k +
                         Gamma_k^n {sum_{j<q} F_k^j} G_k (mirrored), applied
                         as q + 2 mat-vecs, with theta_0 = L_0 b; the error
                         contracts by F_k^q Gamma_k^n per step (eq. riem1) */
  int init_order;     /* h of the initial series, eqs. (g01)-(g03): G_0 =
                         S^-1 sum_{j<h} (I - A S^-1)^j, so F_0 = (I - A S^-1)^h
                         and F_k = F_0^(n^k).  0 or 1: G_0 = S^-1.  Classical
                         and table forms only.                               */
  int init_p, init_w; /* its factorization, h = init_w (init_p + 1); both 0:
                         init_p = h - 1, init_w = 1                           */
  int graph;          /* 1: when the Newton-Schulz phase has a fixed length
                         (floor_detect = 0, f_tol <= 0, no accelerator, a
                         classical or table form, no initial series, timing
                         off), enqueue its k_max steps with their Richardson
                         updates without host round trips, captured once into
                         a HIP graph and replayed on later solves with the same
                         operands and options; the history is recorded on the
                         device and read once.  Otherwise ignored.  Batched
                         submissions: see ns_batch_submit.                  */
} ns_solve_opts;

#define NS_HIST_F 65
#define NS_HIST_R 200

typedef struct {
  int status;            /* NS_OK, NS_EDIVERGED or NS_ENOCONV               */
  int ns_stop;           /* ns_stop_reason of the Newton-Schulz phase        */
  int refine_stop;       /* ns_stop_reason of the refinement phase           */
  int ns_steps;
  int refine_steps;
  int precision;         /* ns_precision the solve ran in                    */
  double alpha;
  double rel_resid;      /* ||b - A theta||_2 / ||b||_2 of the returned theta */
  int64_t mmm;           /* matrix-matrix products executed                  */
  double gemm_flop;      /* 2 n^3 per product                               */
  int n_fnorm;           /* entries of fnorm_hist: ||F_k||_F, k = 0..ns_steps */
  double fnorm_hist[NS_HIST_F];
  int n_resid;           /* entries of resid_hist: relative residual of every
                            theta formed, in order                           */
  double resid_hist[NS_HIST_R];
} ns_solve_report;

/* Coupled solve (eq. redttk1 with omega_k = G_k, Newton-Schulz first in each
 * step): ns_init_scale, theta_0 per theta0_mode, then per step k ns_step and
 * one Richardson update with G_k, then the stop rule on ||F_k||_F; then
 * refinement-only Richardson steps until resid_tol, refine_max or a stall.
 * theta (device, length n) receives the solution.  report may be NULL.
 * Returns NS_OK if resid_tol was reached, NS_ENOCONV if not, NS_EDIVERGED if
 * the iteration diverged (theta is then undefined). */
int richardson_ns_solve(ns_solver* s, const double* b, double* theta,
                        const ns_solve_opts* opts, ns_solve_report* report);

/* ---- Batched solves of many independent systems (uneven sizes) ----------
 *
 * One submission solves `count` independent SPD systems in ONE persistent
 * kernel launch per precision: each workgroup pulls whole systems (largest n
 * first) and runs the complete coupled solve of richardson_ns_solve for each
 * (squaring form of order opts->order, scale ||A||_F or ||A||_inf / 2 + eps,
 * theta_0 = b / alpha).  Products run in float32 MFMA for NS_PREC_FP32; the
 * systems whose float32 solve does not reach opts->resid_tol are re-solved in
 * float64 MFMA by a second launch (report.precision tells which);
 * NS_PREC_FP64 uses float64 only.  Richardson residuals and theta are float64
 * throughout.  A submission whose systems all have n <= 64 (order 2 or 4) runs
 * a kernel that keeps each system's whole iteration in the workgroup's LDS. */
typedef struct ns_batch ns_batch;

/* Device workspace for up to `max_count` systems of size <= max_n, solved by
 * up to `slots` concurrent workgroups (each owns one slot of iterate
 * buffers).  Returns 0 for invalid arguments. */
size_t ns_batch_workspace_bytes(int64_t max_n, int max_count, int slots);

/* Create a batch handle.  precision: NS_PREC_FP32 (with float64 escalation)
 * or NS_PREC_FP64.  max_n <= 4096.  workspace: caller-owned device buffer of
 * >= ns_batch_workspace_bytes(max_n, max_count, slots) bytes, 256-B aligned.
 * Errors: NS_EINVAL, NS_ENOMEM (workspace too small), NS_EHIP. */
int ns_batch_create(int device, void* hip_stream, int64_t max_n, int max_count,
                    int slots, int precision, void* workspace, size_t bytes,
                    ns_batch** out);

/* Launch shape of the float32 (or float64-only) pass: waves per workgroup
 * (1, 2, 4 or 8) and number of workgroups (0: one per slot).  Set by
 * ns_batch_autotune or by the caller.  The float64 pass that re-solves the
 * systems float32 could not runs eight-wave workgroups, one per CU.  The LDS
 * kernel for n <= 64 runs eight waves when waves_per_group is 8, else four. */
int ns_batch_set_launch(ns_batch* b, int waves_per_group, int groups);

/* Float64 re-solve of the systems float32 could not solve: in submissions
 * of at least min_count systems whose largest has n >= 128, the re-solves run
 * in lockstep across the GPU (each product shared by all CUs; a fixed
 * schedule of about 170 launches per submission), otherwise one workgroup
 * per system.  Default 512; 0 turns lockstep off.  Errors: NS_EINVAL. */
int ns_batch_set_lockstep(ns_batch* b, int min_count);

/* Enqueue the solves of `count` systems.  opts->graph = 1: the submission's
 * device work (reset of its counters by a kernel, the persistent kernels) is
 * captured once into a HIP graph and replayed by later submissions with the
 * same systems (pointers, sizes), options and launch shape; any other
 * submission re-captures, and an ordinary submission in between makes the
 * next graph submission re-capture.  Results are identical either way.
 * n, A, lda, b, theta are HOST arrays
 * of length count holding each system's size and DEVICE pointers (A: row-major
 * float64 n x n, lda >= n; b, theta: float64 n).  The caller keeps A, b,
 * theta alive and unmodified (theta: untouched) until ns_batch_poll reports
 * completion.  One submission may be in flight per handle.  Errors:
 * NS_EBUSY (previous ticket not polled to completion), NS_ENOMEM (count >
 * max_count or a system larger than max_n: the admission check), NS_EINVAL
 * (options other than the squaring form of order 2^s, theta0_mode 0; an
 * unknown scale).  Scales: Frobenius, inf / 2, or S = diag(A) (Section 2;
 * a system whose 2S - A is not positive definite diverges and is reported
 * NS_EDIVERGED, its report's alpha = max_i A_ii). */
int ns_batch_submit(ns_batch* b, int count, const int64_t* n, const double* const* A,
                    const int64_t* lda, const double* const* b_vec,
                    double* const* theta, const ns_solve_opts* opts, uint64_t* ticket);

/* Completion of a ticket.  wait = 0: returns NS_EBUSY if the kernel has not
 * finished; wait != 0: blocks.  On completion fills reports[0..count) (host
 * array, may be NULL; fnorm_hist only, no resid_hist) and returns NS_OK if
 * every system reached resid_tol, else NS_ENOCONV (see each report.status). */
int ns_batch_poll(ns_batch* b, uint64_t ticket, int wait, ns_solve_report* reports);

/* Project autotuner: time every launch shape (1, 2, 4, 8 waves per workgroup
 * x 1, 2, 4, 8 workgroups per CU, within the slots) on the given batch (each
 * candidate solves it completely, synchronously), keep the fastest with
 * ns_batch_set_launch and return it.  Same arguments as ns_batch_submit. */
int ns_batch_autotune(ns_batch* b, int count, const int64_t* n, const double* const* A,
                      const int64_t* lda, const double* const* b_vec,
                      double* const* theta, const ns_solve_opts* opts,
                      int* best_waves, int* best_groups, double* best_ms);

/* Per-system timeline of the last ticket returned by ns_batch_poll (a tracing
 * aid for the scheduler): times_us[4 i + 0..3] = begin and end of the float32
 * attempt, begin and end of the float64 attempt of system i (NAN when that
 * attempt did not run), in microseconds from the earliest begin in the batch,
 * read from the device's constant-rate wall clock; workgroup[2 i + 0..1]
 * (optional) = the workgroup that ran each attempt (-1: not run).  Arrays
 * hold 4 x count and 2 x count entries.  Errors: NS_EINVAL (another ticket,
 * NULL times_us), NS_EHIP. */
int ns_batch_timeline(ns_batch* b, uint64_t ticket, double* times_us, int32_t* workgroup);

int ns_batch_destroy(ns_batch* b);

/* ---- Admission by HBM footprint -----------------------------------------
 *
 * A ledger of device bytes in service against a budget, for serving loops
 * that admit requests only while their inputs and workspaces fit (the
 * request loop of the serving workload).  Host memory only; every call is
 * thread-safe (one mutex per ledger), so any number of host threads may admit
 * and release through one ledger. */
typedef struct ns_ledger ns_ledger;

/* budget_bytes > 0.  Errors: NS_EINVAL, NS_ENOMEM (host allocation). */
int ns_ledger_create(size_t budget_bytes, ns_ledger** out);

/* Admit `bytes` if they fit: NS_OK (in service += bytes), NS_ENOMEM if the
 * bytes in service would exceed the budget (nothing changes; retry after a
 * release), NS_EINVAL if `bytes` exceeds the whole budget (never fits). */
int ns_ledger_admit(ns_ledger* l, size_t bytes);

/* Return `bytes` admitted earlier.  NS_EINVAL if more than are in service. */
int ns_ledger_release(ns_ledger* l, size_t bytes);

/* Bytes in service, their peak, the budget, and the numbers of admissions
 * and of NS_ENOMEM refusals so far (any pointer may be NULL). */
int ns_ledger_query(ns_ledger* l, size_t* in_use, size_t* peak, size_t* budget,
                    uint64_t* admitted, uint64_t* refused);
int ns_ledger_destroy(ns_ledger* l);

/* Device bytes one richardson_ns_solve of dimension n holds while it runs:
 * the workspace (ns_workspace_bytes) plus A, b and theta in float64.
 * 0 for invalid arguments. */
size_t ns_solve_footprint(int64_t n, int precision, int composite);

/* Attach a ledger to a batch handle (NULL detaches).  Each ns_batch_submit
 * then admits the submission's footprint, the sum of (n^2 + 2 n) * 8 bytes
 * of its systems' A, b and theta: NS_ENOMEM (over the budget) or NS_EINVAL
 * (larger than the whole budget) is returned with nothing enqueued.
 * ns_batch_poll releases the bytes when it reports completion, and
 * ns_batch_destroy releases a submission still in flight.  Errors:
 * NS_EINVAL, NS_EBUSY (a submission in flight). */
int ns_batch_set_ledger(ns_batch* b, ns_ledger* ledger);

/* Per-kernel timing with HIP events on the solver's stream.  While enabled,
 * every GEMM launch is bracketed by an event pair.  ns_timing_read returns
 * the number of timed GEMM launches, their summed duration (ms) and their
 * summed algorithmic flop (2 m n k each) since the last reset, synchronizing
 * the stream.  kind: 0 = all GEMMs, 1 = float64 GEMMs, 2 = float32,
 * 3 = bf16, 4 = split half-precision (the interval includes the operand
 * split passes). */
int ns_timing_enable(ns_solver* s, int enable);
int ns_timing_read(ns_solver* s, int kind, int64_t* launches, double* total_ms,
                   double* flop);
int ns_timing_reset(ns_solver* s);

/* GEMM flags. */
#define NS_GEMM_SYMMETRIC 1 /* symmetric output (m == n): only the tiles on
                               or above the diagonal are computed from X Y
                               (+ addends); the lower triangle is written as
                               their mirror, so D is exactly symmetric.  Valid
                               when X Y + E1 + E2 is symmetric in exact
                               arithmetic (every product of the iteration is a
                               polynomial in A). */

/* Kernel-level entry point (tests, benchmarks): one float64 MFMA GEMM with
 * the solver's fused epilogue,
 *   D = diag * I + scale * (X Y) + E1 + E2,       X: m x k, Y: k x n,
 * E1 / E2 optional (NULL), row-major device float64 with leading dimensions.
 * flags: 0 or NS_GEMM_SYMMETRIC.  D must not alias X or Y.  If sumsq_out is
 * non-NULL it must point to 1 + ns_gemm_f64_partials(m, n, flags) device
 * doubles: sumsq_out[0] receives sum(D_ij^2) over the whole output, reduced
 * in a fixed order, the rest is scratch for per-tile partial sums.
 * Enqueued on hip_stream; does not synchronize.  Errors: NS_EINVAL
 * (negative size, NULL operand, ld too small, D aliasing X or Y, unknown
 * flags, symmetric with m != n), NS_EHIP (launch failure). */
int ns_gemm_f64(void* hip_stream, int64_t m, int64_t n, int64_t k,
                const double* X, int64_t ldx, const double* Y, int64_t ldy,
                double* D, int64_t ldd, const double* E1, int64_t lde1,
                const double* E2, int64_t lde2, double diag, double scale,
                int flags, double* sumsq_out);

/* Upper bound on the per-tile partial sums ns_gemm_f64 / ns_gemm_f64_ws
 * write for an m x n output. */
int64_t ns_gemm_f64_partials(int64_t m, int64_t n, int flags);

/* ns_gemm_f64 with caller-owned device scratch.  When the output tiles do not
 * fill a whole number of rounds of resident workgroups, the tiles of the last,
 * partial round can be cut along K into slices computed by otherwise idle
 * workgroups and summed, in a fixed order, by a second kernel; that needs
 * ns_gemm_f64_scratch_bytes(m, n, k, flags) bytes of scratch (0: no split for
 * this shape on this device).  With less scratch (or NULL) the call is exactly
 * ns_gemm_f64.  The scratch (8-byte aligned) is used only while the call's
 * kernels run on hip_stream; concurrent calls need separate scratch.  The
 * result equals ns_gemm_f64's up to the summation order over K.  Errors as
 * ns_gemm_f64, plus NS_EINVAL for misaligned scratch. */
size_t ns_gemm_f64_scratch_bytes(int64_t m, int64_t n, int64_t k, int flags);
int ns_gemm_f64_ws(void* hip_stream, int64_t m, int64_t n, int64_t k,
                   const double* X, int64_t ldx, const double* Y, int64_t ldy,
                   double* D, int64_t ldd, const double* E1, int64_t lde1,
                   const double* E2, int64_t lde2, double diag, double scale,
                   int flags, void* scratch, size_t scratch_bytes,
                   double* sumsq_out);

/* Kernel-level entry points of the float32 and bf16 MFMA GEMMs used by the
 * float32 and mixed modes (tests, benchmarks), with the same fused epilogue
 * computed in float32:
 *   ns_gemm_f32:      D = diag I + scale (X Y)   + E1 + E2,  X: m x k, Y: k x n
 *   ns_gemm_bf16_nt:  D = diag I + scale (X Y^T) + E1 + E2,  X: m x k, Y: n x k
 * X / Y are row-major device float32 (ns_gemm_f32) or bf16 stored as raw
 * 16-bit patterns (ns_gemm_bf16_nt); accumulation is float32.  D (float32)
 * and Db (bf16 copy of D, rounded to nearest even) are optional but not both
 * NULL; E1, E2 are optional float32 addends.  Outputs must not alias X or Y.
 * sumsq_out, when non-NULL, must hold 1 + ns_gemm_lp_partials(m, n) device
 * doubles; [0] receives sum(D_ij^2) accumulated in float64 in a fixed order.
 * Enqueued on hip_stream; no synchronization.  Errors as ns_gemm_f64. */
int ns_gemm_f32(void* hip_stream, int64_t m, int64_t n, int64_t k,
                const float* X, int64_t ldx, const float* Y, int64_t ldy,
                float* D, int64_t ldd, uint16_t* Db, int64_t lddb,
                const float* E1, int64_t lde1, const float* E2, int64_t lde2,
                float diag, float scale, double* sumsq_out);
int ns_gemm_bf16_nt(void* hip_stream, int64_t m, int64_t n, int64_t k,
                    const uint16_t* X, int64_t ldx, const uint16_t* Y, int64_t ldy,
                    float* D, int64_t ldd, uint16_t* Db, int64_t lddb,
                    const float* E1, int64_t lde1, const float* E2, int64_t lde2,
                    float diag, float scale, double* sumsq_out);

/* Number of per-tile partial sums ns_gemm_f32 / ns_gemm_bf16_nt /
 * ns_gemm_bf16_nt_ws / ns_gemm_f32_split write. */
int64_t ns_gemm_lp_partials(int64_t m, int64_t n);

/* ns_gemm_bf16_nt with flags and caller-owned device scratch.
 * NS_GEMM_SYMMETRIC is currently DISABLED (NS_EINVAL, and
 * ns_gemm_bf16_scratch_bytes returns 0): its kernel faulted the GPU on its
 * first test and the cause has not been found.  Without flags the call is
 * ns_gemm_bf16_nt.  Intended behaviour with NS_GEMM_SYMMETRIC (m == n; X Y^T + E1 + E2 symmetric in exact arithmetic,
 * as every power and assembly product of the iteration is) only the
 * 128 x 128 tiles on or above the diagonal are computed and the lower
 * triangle is written as their mirror, so D and Db are exactly symmetric.
 * When those tiles leave a partial last round of resident workgroups, that
 * round is cut along K into slices stored in the scratch and summed in a
 * fixed order by a second kernel.  Shapes where this does not save at least
 * 10% run the full-output kernel (the result is then X Y^T in full, not
 * mirrored).  scratch: ns_gemm_bf16_scratch_bytes(m, n, k, flags) bytes
 * (0: none needed), 16-byte aligned.  Errors as ns_gemm_bf16_nt, plus
 * NS_ENOMEM for too little scratch and NS_EINVAL for m != n with the flag. */
size_t ns_gemm_bf16_scratch_bytes(int64_t m, int64_t n, int64_t k, int flags);
int ns_gemm_bf16_nt_ws(void* hip_stream, int64_t m, int64_t n, int64_t k,
                       const uint16_t* X, int64_t ldx, const uint16_t* Y, int64_t ldy,
                       float* D, int64_t ldd, uint16_t* Db, int64_t lddb,
                       const float* E1, int64_t lde1, const float* E2, int64_t lde2,
                       float diag, float scale, int flags, double* sumsq_out,
                       void* scratch, size_t scratch_bytes);

/* float32-class product on the half-precision matrix cores: the operation,
 * operands and outputs of ns_gemm_f32 (D = diag I + scale (X Y) + E1 + E2,
 * X: m x k, Y: k x n, row-major float32), computed from split operands.
 * Each operand is scaled by a power of two 2^e that brings its largest
 * magnitude into [2^14, 2^15) and written as two IEEE half-precision planes,
 * hi = half(x 2^e) and lo = half(x 2^e - hi) (22 significant bits; Y is
 * stored transposed); the product is hi hi + hi lo + lo hi with float32
 * accumulation (v_mfma_f32_32x32x16_f16), scaled back by 2^-(ex + ey).
 * Error: float32 accumulation plus operand rounding below 2^-21 relative
 * (2^-24 for float32 operands).  Scale exponents are clamped to [-100, 100];
 * entries below 2^-24 of the largest magnitude lose relative accuracy (half
 * subnormals), and a non-finite operand gives non-finite outputs.
 * The mixed-precision solver uses this product for the residual, the
 * G-side update and the composite merge (NS_PREC_MIXED_SPLIT).
 * scratch: device memory of ns_gemm_f32_split_scratch_bytes(m, n, k) bytes,
 * 256-byte aligned, used only by the work this call enqueues (calls that
 * share it must be ordered on one stream).  NS_ENOMEM if smaller, NS_EINVAL
 * if misaligned; other errors as ns_gemm_f32. */
size_t ns_gemm_f32_split_scratch_bytes(int64_t m, int64_t n, int64_t k);
int ns_gemm_f32_split(void* hip_stream, int64_t m, int64_t n, int64_t k,
                      const float* X, int64_t ldx, const float* Y, int64_t ldy,
                      float* D, int64_t ldd, uint16_t* Db, int64_t lddb,
                      const float* E1, int64_t lde1, const float* E2, int64_t lde2,
                      float diag, float scale, double* sumsq_out,
                      void* scratch, size_t scratch_bytes);

/* ---- Tile table of the project's tile autotuner --------------------------
 *
 * The MFMA GEMMs pick their output tile by a rule fitted on MI355X
 * (occupancy of the 256 compute units per tile round).  A tile autotuner
 * (autotune.tune_tiles in the Python package: it times each candidate tile
 * per family and size and keeps the fastest) overrides that rule per GEMM
 * family and size bucket: products whose output is m x n use the tile set
 * for bucket ceil(log2(max(m, n))).  Families: NS_TILE_F64 (ns_gemm_f64 and
 * the float64 solver products; tiles 64, 128, 256: the 256 x 128 tile serves
 * full-output products with K a multiple of 16, N even, even leading
 * dimensions and 16-byte aligned X and Y; symmetric-output products and
 * other shapes then take the rule's choice of 64 or 128), NS_TILE_F32 (float32 MFMA;
 * 64, 128, 256: the 256 tile needs K a multiple of 32, N a multiple of 4 and
 * 16-byte aligned rows, and falls back to 128 otherwise), NS_TILE_BF16 (bf16
 * powers; 64, 128, 256), NS_TILE_F16S (split half-precision products; 64,
 * 128, 256).  Tile 0 restores the rule.  The
 * table is process-wide (all devices); every tile is valid for every shape,
 * and buffers sized by ns_gemm_f64_partials / ns_gemm_lp_partials /
 * ns_workspace_bytes hold the partial sums of any choice.  Setting an entry
 * while products run on other threads is allowed (each launch reads it
 * once).  ns_tile_set errors: NS_EINVAL (unknown family, bucket outside
 * 0..23, or a tile the family does not have).  ns_tile_get returns the
 * entry, or -1 for invalid arguments. */
#define NS_TILE_F64 0
#define NS_TILE_F32 1
#define NS_TILE_BF16 2
#define NS_TILE_F16S 3
int ns_tile_set(int family, int log2_dim, int tile);
int ns_tile_get(int family, int log2_dim);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, allocation-free serving loops, harnesses that forbid hipMalloc):
 * ns_gemm_f32_split without the scratch argument.  The split planes, block
 * maxima, scale exponents and per-tile partial sums live in a scratch array
 * built into the library, one copy per GPU, of NS_SPLIT_NOALLOC_MAX_BYTES
 * bytes, held from the library's load until the process ends; the call makes
 * no allocation of any kind.  sumsq_out, when non-NULL, is ONE device double
 * that receives sum(D_ij^2) (the partial sums stay in the built-in array).
 * Shapes need ns_gemm_f32_split_scratch_bytes(m, n, k) bytes, plus
 * 8 ns_gemm_lp_partials(m, n) rounded up to 256 with sumsq_out; larger shapes
 * are rejected with NS_ENOMEM (square shapes up to about n = 2800 fit).
 * Every call on a GPU shares that GPU's array and leaves its contents behind:
 * calls that overlap in time on one GPU (different streams, or several host
 * threads) race and must be serialised by the caller.  Nothing in the array
 * needs to start at zero: every byte a call reads was written earlier by the
 * same call.  Operation, arguments, results and other errors as
 * ns_gemm_f32_split; the stream must belong to the current device. */
#define NS_SPLIT_NOALLOC_MAX_BYTES (64u << 20)
int ns_gemm_f32_split_noalloc(void* hip_stream, int64_t m, int64_t n, int64_t k,
                              const float* X, int64_t ldx, const float* Y, int64_t ldy,
                              float* D, int64_t ldd, uint16_t* Db, int64_t lddb,
                              const float* E1, int64_t lde1, const float* E2, int64_t lde2,
                              float diag, float scale, double* sumsq_out);

const char* ns_status_string(int status);
const char* ns_last_error(void);

/* Library version string. */
const char* ns_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NSR_H */
