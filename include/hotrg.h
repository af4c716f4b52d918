/*
 * hotrg.h -- C ABI of libhotrg.so: the HOTRG coarse-graining step on the 2D
 * square lattice (arXiv 2306.00358, Sec. 2 and Fig. 1) on one AMD MI355X
 * (gfx950) GPU.
 *
 * Plain C99.  No C++ types or exceptions cross this boundary.  Pointers are
 * host pointers unless the argument is documented as a device pointer.
 * Every function returns a hotrg_status; on error the outputs are left
 * untouched and hotrg_last_error() returns a message (per calling thread).
 *
 * Site tensors are rank 4 with legs (left, up, right, down), stored
 * row-major with the left leg slowest: T[l][u][r][d].  A *directional step*
 * merges two vertically adjacent copies (first above second) and fuses the
 * pair of left legs (second.left, first.left) -- and likewise the right
 * pair -- into one leg of dimension D' = min(d_cut, Dx*Dx), where Dx is the
 * left/right dimension and Dy the up/down dimension before the step.  After
 * the step the legs are transposed, (l,u,r,d) -> (u,l,d,r), so the next step
 * coarse-grains the orthogonal direction; two directional steps make one
 * iteration of the paper, and K steps cover 2^K sites.
 *
 * Per step k the tensor is divided by n_k = max|T| and
 *     ln Z / N = ln n_0 + sum_k 2^-k ln n_k + 2^-K ln sum_{i,j} T_K[i][j][i][j]
 * (periodic boundary conditions, Sec. 2).  The environment eigensolver and
 * this accumulation are always FP64; `prec` selects the arithmetic of the
 * contractions only.
 */
#ifndef HOTRG_H
#define HOTRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HOTRG_OK = 0,
  HOTRG_ERR_INVALID = 1,   /* bad argument: sizes, model, d_cut < 1, null pointer */
  HOTRG_ERR_OOM = 2,       /* the request does not fit the context's HBM budget */
  HOTRG_ERR_DEVICE = 3,    /* a HIP / rocSOLVER call failed */
  HOTRG_ERR_NUMERIC = 4,   /* non-finite norm, eigensolver failure, trace <= 0 */
  HOTRG_ERR_NOT_READY = 5, /* submitted request still running */
  HOTRG_ERR_CANCELLED = 6  /* submitted request was cancelled */
} hotrg_status;

typedef enum {
  HOTRG_ISING = 0, /* Ising, bond dimension 2 (Sec. 3.2) */
  HOTRG_XY = 1,    /* classical XY, character expansion, |n| <= n_max (Sec. 3.1, Delta = 1) */
  HOTRG_POTTS = 2, /* q-state Potts, Cholesky split of the bond weight (Sec. 3.3) */
  HOTRG_RAW = 3,   /* caller-supplied initial tensor */
  HOTRG_GXY = 4    /* generalized XY, Eq. (gXY_ham) with h = 0 (Sec. 3.1): bond weight
                      exp(beta Delta cos x + beta (1 - Delta) cos 2x) with character
                      coefficients c_n = sum_m I_{n-2m}(beta Delta) I_m(beta (1 - Delta)),
                      charges |n| <= n_max */
} hotrg_model;

typedef enum {
  HOTRG_FP64 = 0,      /* FP64 MFMA contractions */
  HOTRG_FP32 = 1,      /* FP32 MFMA contractions, FP32 intermediates */
  HOTRG_BF16X3 = 2,    /* split-BF16, three products, FP32 accumulation */
  HOTRG_PREC_AUTO = 3  /* whole runs only (hotrg_run, batch, submit): the precision
                          with the least estimated time whose a-priori error bound
                          (hotrg_opts.tol) is met; needs tol > 0 */
} hotrg_precision;

typedef enum {
  HOTRG_TRUNC_PLAIN = 0,   /* keep the first D' eigenvectors (the paper) */
  HOTRG_TRUNC_MULTIPLET = 1 /* never split a cluster of eigenvalues closer than
                               degen_tol * lambda_1 at the cut: the cluster is
                               dropped whole and U is padded with zero columns */
} hotrg_trunc;

typedef enum {
  HOTRG_EIG_AUTO = 0,  /* block subspace iteration (FP64, Rayleigh-Ritz) when
                          D' is small against dx*dx, dense solver otherwise or
                          if the iteration does not converge */
  HOTRG_EIG_DENSE = 1  /* always the dense FP64 solver (rocSOLVER dsyevd) */
} hotrg_eig;

typedef enum {
  HOTRG_ISO_ONE_SIDED = 0, /* the projector comes from the environment of the left
                              pair of legs and truncates both pairs (Sec. 2) */
  HOTRG_ISO_TWO_SIDED = 1  /* original HOTRG: the projectors of the left and of the
                              right environment are both formed and the one with the
                              smaller truncation error is used; the right one only
                              when smaller by more than 1e-12, so reflection-symmetric
                              models keep the one-sided result.  FP64 contractions
                              only (HOTRG_ERR_INVALID otherwise); about twice the
                              environment and eigensolver work */
} hotrg_isometry;

typedef struct {
  int model;          /* hotrg_model */
  double beta;        /* inverse temperature 1/T (k_B = 1) */
  double J;           /* Ising coupling (J * beta >= 0); ignored otherwise */
  int n_max;          /* XY: charges |n| <= n_max, bond dimension 2 n_max + 1 */
  int q;              /* Potts: number of states, >= 2 */
  const double* raw;  /* HOTRG_RAW: host array raw_dx*raw_dy*raw_dx*raw_dy,
                         legs (l,u,r,d); copied during the call */
  int raw_dx, raw_dy; /* HOTRG_RAW: left/right and up/down dimensions */
  double delta;       /* GXY: weight Delta of cos(theta_i - theta_j), 0 <= Delta <= 1
                         (1 - Delta weighs cos 2(theta_i - theta_j)); ignored otherwise */
} hotrg_model_params;

typedef struct {
  int d_cut;          /* kept bond dimension, >= 1 */
  int n_steps;        /* directional steps for hotrg_run, >= 0 */
  int prec;           /* hotrg_precision */
  int trunc;          /* hotrg_trunc */
  double degen_tol;   /* multiplet tolerance tau (relative to lambda_1) */
  int spec_len;       /* spectrum values recorded per step (0: none) */
  int eig;            /* hotrg_eig: how the leading eigenpairs of M are found */
  int isometry;       /* hotrg_isometry */
  double tol;         /* reduced precision: target relative error of ln Z/N against
                         the FP64 result (0: none).  Step k's contractions add at
                         most C_p 2^-k to it (C_FP32 = 2e-5, C_BF16X3 = 1e-4: 2.5x the largest
                         measured on the Ising and XY workloads; ln Z/N weighs step k by 2^-k,
                         Sec. 2), so steps before k0 = ceil(1 + log2(C_p / tol)) keep
                         FP64 contractions; the bound of the steps actually reduced
                         is returned in hotrg_result.err_bound */
} hotrg_opts;

typedef struct {
  int dx, dy;         /* dimensions before the step */
  int d_new;          /* D' = min(d_cut, dx*dx) */
  int kept;           /* columns of U that are not zero padding */
  double log_norm;    /* ln n_k */
  double trunc_err;   /* 1 - sum_{m<=kept} lambda_m / trace(M) */
  double cut_gap;     /* (lambda_{D'} - lambda_{D'+1}) / lambda_1; -1 when nothing is cut */
  double lnz_torus;   /* ln Z / N of the 2^k-site torus after this step */
  int side;           /* environment the projector came from: 0 left, 1 right */
} hotrg_step_info;

typedef struct {
  double lnz_per_site;     /* ln Z / N */
  int n_steps;             /* steps done */
  hotrg_step_info* steps;  /* caller-owned array of n_steps entries, or NULL */
  double* spectra;         /* caller-owned [n_steps][spec_len] lambda/lambda_1
                              descending (zero past dx*dx), or NULL */
  double seconds;          /* wall time of the run itself */
  double t_submit, t_start, t_end; /* submitted requests: host times in seconds
                                      since the context was created */
  int prec_used;           /* precision the result was computed with (a
                              submitted reduced-precision problem that fails
                              with HOTRG_ERR_NUMERIC is re-run once in FP64) */
  double err_bound;        /* a-priori bound on the relative ln Z/N error against
                              the FP64 result: C_p sum_{reduced steps k} 2^-k
                              (0 for FP64) */
} hotrg_result;

typedef struct hotrg_ctx hotrg_ctx;
typedef struct hotrg_state hotrg_state;

/* Context on one GPU.  `hip_stream` is a hipStream_t to run on (borrowed, may
 * be NULL for a stream of the context's own).  `hbm_budget` bounds the
 * device memory the context may hold, in bytes (0: no bound).  The context
 * owns all device buffers and states it creates.  Not thread-safe except for
 * the submit/poll/wait/cancel family. */
hotrg_status hotrg_ctx_create(int device, void* hip_stream, size_t hbm_budget, hotrg_ctx** out);
void hotrg_ctx_destroy(hotrg_ctx* ctx);
const char* hotrg_last_error(void);
size_t hotrg_ctx_bytes_in_use(const hotrg_ctx* ctx);

/* Build the initial tensor of `params` in FP64 on the host, upload it
 * and divide it by n_0 = max|T0| (Sec. 3: Ising, XY, Potts tensors).  The
 * state records ln n_0 and is owned by ctx until hotrg_state_free. */
hotrg_status hotrg_init_tensor(hotrg_ctx* ctx, const hotrg_model_params* params,
                               int prec, hotrg_state** out);

/* One directional coarse-graining step (Sec. 2, Fig. 1): environment
 * M, FP64 eigendecomposition, projector U, the three contractions, the
 * transposition of legs and the normalisation.  `info` (may be NULL)
 * receives the step record and `spectrum` (host, may be NULL) the first
 * opts->spec_len values of lambda/lambda_1; either being non-NULL makes the
 * call wait for the GPU.  opts->n_steps is ignored. */
hotrg_status hotrg_step(hotrg_ctx* ctx, hotrg_state* st, const hotrg_opts* opts,
                        hotrg_step_info* info, double* spectrum);

/* ln Z / N from the steps done so far and the periodic trace. */
hotrg_status hotrg_finish(hotrg_ctx* ctx, hotrg_state* st, double* lnz_per_site);

/* Copy the current (normalised) tensor to the host.  `dims` receives
 * (dx, dy); `cap` is the capacity of `host` in doubles; `acc` receives
 * ln n_0 + sum_k 2^-k ln n_k and `k` the number of steps done. */
hotrg_status hotrg_state_export(hotrg_ctx* ctx, const hotrg_state* st, double* host, size_t cap,
                                int dims[2], double* acc, int* k);
void hotrg_state_free(hotrg_ctx* ctx, hotrg_state* st);

/* Init, opts->n_steps directional steps, finish; one host wait at the
 * end.  result->steps / result->spectra are filled when non-NULL. */
hotrg_status hotrg_run(hotrg_ctx* ctx, const hotrg_model_params* params, const hotrg_opts* opts,
                       hotrg_result* result);

/* ---- many problems: batch and serving loop ------------------------------
 * The context runs submitted problems on a pool of workers, each with its
 * own HIP stream and device workspace, so problems overlap on the GPU.  A
 * queued problem is admitted when a worker is free and its estimated
 * device footprint fits the HBM budget (the context's hbm_budget, or 90% of
 * the free device memory when that is 0) next to the running ones; a problem
 * that can never fit fails with HOTRG_ERR_OOM.  A problem's result does not
 * depend on what runs beside it (same kernels, same order).  A problem with
 * FP32 / split-BF16 contractions that ends with HOTRG_ERR_NUMERIC (e.g. a
 * non-positive final trace after reduced-precision noise has driven the
 * flow away) is queued once more with FP64 contractions; prec_used says
 * which precision produced the result.
 * submit/poll/wait/cancel are thread-safe. */

/* Worker count (default 16); takes effect before the first submit or batch. */
hotrg_status hotrg_ctx_set_workers(hotrg_ctx* ctx, int n_workers);

/* Queue one problem.  `result` is caller-owned and must stay valid (with its
 * steps/spectra arrays, if set) until the problem completes or is cancelled;
 * the raw tensor of HOTRG_RAW is copied during the call. */
hotrg_status hotrg_submit(hotrg_ctx* ctx, const hotrg_model_params* params, const hotrg_opts* opts,
                          hotrg_result* result, uint64_t* ticket);
/* HOTRG_ERR_NOT_READY while queued or running; afterwards the problem's own
 * status (HOTRG_OK, an error, or HOTRG_ERR_CANCELLED).  A finished ticket
 * stays valid until hotrg_release or the context's destruction. */
hotrg_status hotrg_poll(hotrg_ctx* ctx, uint64_t ticket);
/* Wait up to timeout_s seconds (< 0: no limit); returns as hotrg_poll. */
hotrg_status hotrg_wait(hotrg_ctx* ctx, uint64_t ticket, double timeout_s);
/* Cancel a queued problem, or stop a running one at its next step boundary. */
hotrg_status hotrg_cancel(hotrg_ctx* ctx, uint64_t ticket);
/* Forget a finished ticket: its record (and the copy of a HOTRG_RAW tensor)
 * is freed and later calls with it return HOTRG_ERR_INVALID.
 * HOTRG_ERR_NOT_READY while the problem is queued or running.  A serving
 * loop releases every ticket it has read, so the context's bookkeeping stays
 * bounded; hotrg_run_batch releases its own. */
hotrg_status hotrg_release(hotrg_ctx* ctx, uint64_t ticket);
/* The precision schedule hotrg_run would use (host arithmetic, no GPU):
 * `prec` the precision of the reduced steps (HOTRG_PREC_AUTO resolved;
 * HOTRG_FP64 when none), `first_reduced` the first step allowed to be
 * reduced (steps before the steady state are FP64 regardless), `err_bound`
 * the a-priori relative error bound of hotrg_result.err_bound.  Any output
 * may be NULL. */
hotrg_status hotrg_plan(const hotrg_model_params* params, const hotrg_opts* opts, int* prec,
                        int* first_reduced, double* err_bound);
/* Estimated peak device bytes of one problem (the admission footprint). */
hotrg_status hotrg_footprint(const hotrg_model_params* params, const hotrg_opts* opts,
                             size_t* bytes);
/* Run n problems on the worker pool and wait for all; `statuses` (may be
 * NULL) receives each problem's status; returns the first failure or OK. */
hotrg_status hotrg_run_batch(hotrg_ctx* ctx, int n, const hotrg_model_params* params,
                             const hotrg_opts* opts, hotrg_result* results,
                             hotrg_status* statuses);

/* Run n problems in lockstep on the context's own stream (the paper's
 * studies scan many temperatures and couplings, Sec. 3.1-3.3): every problem
 * takes its warm-up steps alone, then all of them advance one steady-state
 * directional step per sweep, each phase of the sweep one launch over every
 * problem -- grouped MFMA GEMMs reading a device table of the problems'
 * products (uneven D_cut and shapes), a batched block eigensolver (subspace
 * iteration with a fixed budget of rounds, Rayleigh-Ritz by Householder
 * reduction and divide and conquer, one workgroup per problem; environments of
 * at most 128 rows diagonalised whole by the same two kernels), batched
 * bookkeeping -- and the whole
 * sweep is captured once as a HIP graph and replayed (captured again when a
 * problem has finished its steps).  Grouped launches pick their tile shapes by
 * timing the candidates on the first sweep of a set of shapes.  A problem
 * joins the batch when its steady state has D' + 17 <= p <= 128 and 4p <= D'^2
 * (p = the eigensolver's block size, about 2 D') or D'^2 <= 128 (all problems
 * of a batch alike in this), the one-sided isometry, the
 * automatic eigensolver choice and the batch's steady precision; other
 * problems run whole, one after another, before the batch.  A problem whose
 * batched eigensolve does not converge within the budget is run again alone.
 * Results are as hotrg_run's (to rounding: another summation order).  `results`
 * and `statuses` as for hotrg_run_batch; returns the first failure or OK. */
hotrg_status hotrg_run_grouped(hotrg_ctx* ctx, int n, const hotrg_model_params* params,
                               const hotrg_opts* opts, hotrg_result* results,
                               hotrg_status* statuses);
/* Counters of hotrg_run_grouped on this context: sweeps run, of them graph
 * replays, graph captures, problems re-run alone. */
hotrg_status hotrg_ctx_group_stats(hotrg_ctx* ctx, uint64_t* sweeps, uint64_t* replays,
                                   uint64_t* captures, uint64_t* fallbacks);

/* Internal energy and specific heat per site by finite differences of ln Z/N
 * in beta (Sec. 3.3 obtains the specific heat as a finite-difference second
 * derivative of ln Z): the problem of `params` / `opts` is run at
 * beta + j dbeta, j = -2 .. 2, on the context's worker pool, and the
 * five-point central stencils (error O(dbeta^4)) give
 *   out[0] = ln Z / N at beta,
 *   out[1] = u = -d(ln Z/N)/d beta       (energy per site),
 *   out[2] = c = beta^2 d^2(ln Z/N)/d beta^2   (specific heat per site, k_B = 1).
 * `out` is caller-owned (3 doubles).  HOTRG_ERR_INVALID for HOTRG_RAW, for
 * dbeta <= 0 or beta - 2 dbeta < 0; otherwise the first failing run's status. */
hotrg_status hotrg_thermo(hotrg_ctx* ctx, const hotrg_model_params* params,
                          const hotrg_opts* opts, double dbeta, double* out);
/* Serving counters: requests admitted, queue passes where the oldest queued
 * request did not fit, peak bytes reserved by running requests. */
hotrg_status hotrg_ctx_sched_stats(hotrg_ctx* ctx, uint64_t* admitted, uint64_t* stalls,
                                   size_t* peak_reserved);

/* ---- per-phase timing (HIP events on the context's stream) -------------
 * When enabled, every phase of every step is bracketed by HIP events;
 * hotrg_ctx_timings waits for the stream, copies up to `cap` records into
 * `out` (host) and clears the list.  It returns the number of records
 * copied, or -1 on error. */
enum {
  HOTRG_PHASE_ENV = 0,   /* environment halves, combine, symmetrise */
  HOTRG_PHASE_EIGH = 1,  /* FP64 leading eigenpairs of M */
  HOTRG_PHASE_PROJ = 2,  /* spectrum, truncation, projector layouts */
  HOTRG_PHASE_C1 = 3,    /* X1 = U T */
  HOTRG_PHASE_C2 = 4,    /* X2 = X1 T: the O(D^7) contraction */
  HOTRG_PHASE_C3 = 5,    /* T~ = X2 U, with max|T~| */
  HOTRG_PHASE_NORM = 6   /* log-norm, trace, next operands */
};
typedef struct {
  int step;   /* 1-based step index within its state */
  int phase;  /* HOTRG_PHASE_* */
  int dx, dy, d_new;
  float ms;   /* elapsed time between the phase's events */
} hotrg_phase_time;
hotrg_status hotrg_ctx_enable_timing(hotrg_ctx* ctx, int on);
int hotrg_ctx_timings(hotrg_ctx* ctx, hotrg_phase_time* out, int cap);

/* ---- eigensolver diagnostic ----------------------------------------------
 * The context's last solve for the leading eigenpairs of an environment
 * (Sec. 2; by the last step of hotrg_step / hotrg_run or by
 * hotrg_projector): *sweeps = the block subspace sweeps it took and *resid =
 * the largest relative Ritz residual of the pairs it needed, or *sweeps = 0
 * when the solve was dense (rocSOLVER dsyevd, including a fallback after a
 * block solve that did not converge).  Host pointers, either may be NULL;
 * HOTRG_ERR_INVALID for a NULL ctx. */
hotrg_status hotrg_ctx_last_eig(hotrg_ctx* ctx, int* sweeps, double* resid);

/* ---- primitive contractions on caller device buffers (same kernels) -----
 * All pointers are device pointers of FP64 arrays, row-major; `prec`
 * selects the arithmetic of the contractions (inputs are rounded to it,
 * results are returned as FP64).  They wait for the context's stream. */

/* Environment: M[(i,j),(k,l)] = sum T[j,a,b,e] T[i,e,c,d] T[l,a,b,f] T[k,f,c,d]
 * (Sec. 2), T of shape (dx,dy,dx,dy), M of shape (dx*dx, dx*dx). */
hotrg_status hotrg_environment(hotrg_ctx* ctx, int prec, const double* T, int dx, int dy,
                               double* M);

/* Projector of a step (Sec. 2): the leading eigenpairs of the environment M
 * (device, n x n row-major, symmetric positive semidefinite; not modified)
 * by the step's FP64 eigensolver -- block subspace iteration with
 * Rayleigh-Ritz when d_new is small against n (n >= 1024), else the dense
 * solver -- and the step's truncation rule (`trunc`: hotrg_trunc; with
 * HOTRG_TRUNC_MULTIPLET the cut moves down while the gap at it is at most
 * degen_tol lambda_1).  U (device, n x d_new row-major) receives the
 * eigenvectors of the d_new largest eigenvalues as columns, in descending
 * order (signs as the solver returns them), columns from *kept on zero;
 * spec (host, spec_len values, may be NULL when spec_len = 0) the spectrum
 * lambda_m / lambda_1, descending; *kept (host) the columns kept; *trunc_err
 * (host) 1 - sum_{m < kept} lambda_m / Tr M.  2 <= n, 1 <= d_new <= n.
 * HOTRG_ERR_NUMERIC when the eigensolver does not converge.  Waits for the
 * context's stream. */
hotrg_status hotrg_projector(hotrg_ctx* ctx, const double* M, int n, int d_new, int trunc,
                             double degen_tol, int spec_len, double* U, double* spec, int* kept,
                             double* trunc_err);

/* Coarse tensor: Tt[i,j,k,l] = sum U[a,b,i] T[b,j,d,c] T[a,c,e,l] U[e,d,k]
 * (Sec. 2), T (dx,dy,dx,dy), U (dx,dx,dn), Tt (dn,dy,dn,dy); *max_abs
 * (device, may be NULL) receives max|Tt|. */
hotrg_status hotrg_coarse(hotrg_ctx* ctx, int prec, const double* T, const double* U, int dx,
                          int dy, int dn, double* Tt, double* max_abs);

/* ---- allocation-free coarse contraction ---------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops and harnesses that forbid hipMalloc.  Computes the
 * same T~ and max|T~| as hotrg_coarse with prec = HOTRG_FP64 (C1 -> C2 -> C3
 * with the fixed tile rule instead of the autotuner's choice, so the two may
 * differ in the last bits), but calls no hipMalloc / hipFree / allocating
 * library routine, records no memset, and does not wait: the work is
 * enqueued on the context's stream (the stream given to hotrg_ctx_create,
 * which the caller may be capturing) and the caller synchronises it.
 * All intermediates live in one static device array of
 * HOTRG_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends; every call on a GPU shares that GPU's array, so
 * calls that overlap on one GPU (other streams, other contexts, other
 * threads) race and must be serialised by the caller.  Sizes must satisfy
 *   2 dn dx^2 dy^2 + 3 dx^2 dy^2 + 2 dx^2 dn + 288  <=  scratch bytes / 8
 * (each of the seven buffers is rounded up to 32 doubles; dx = dy = dn = 20
 * fits); larger sizes fail with HOTRG_ERR_INVALID and a
 * message giving the bytes needed.  T, U, Tt and max_abs (may be NULL) are
 * device pointers with the layouts of hotrg_coarse; 1 <= dn <= dx*dx. */
#define HOTRG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
hotrg_status hotrg_coarse_noalloc(hotrg_ctx* ctx, const double* T, const double* U, int dx,
                                  int dy, int dn, double* Tt, double* max_abs);

#ifdef __cplusplus
}
#endif

#endif /* HOTRG_H */
