/*
 * chfsi.h - C ABI of the MI355X (gfx950) Chebyshev-filtered subspace
 * iteration library.
 *
 * The library solves the dense Hermitian generalized eigenproblem
 *     H x = lambda S x      (H Hermitian, S Hermitian positive definite)
 * for the nev smallest eigenpairs, following Algorithm 1 of Berljafa & Di
 * Napoli, "A Parallel and Scalable Iterative Solver for Sequences of Dense
 * Eigenproblems Arising in FLAPW" (arXiv 1305.5120): reduction to standard
 * form (Section 3), a Lanczos estimate of the spectrum's upper end, then
 * repeated Chebyshev filtering (eq. (2)), QR re-orthonormalization,
 * Rayleigh-Ritz and locking of converged pairs.  Solving a sequence of
 * correlated problems (Section 2) warm-starts each solve from the previous
 * solution, which the context keeps on the device.
 *
 * Conventions for every entry point
 *   - complex numbers are complex128: two IEEE doubles (re, im), 16 bytes,
 *     the layout of C99 `double _Complex`, `hipDoubleComplex` and
 *     torch.complex128;
 *   - matrices are column-major with a leading dimension `ld* >= rows`;
 *     H and S are read in full (S only in its lower triangle);
 *   - pointers documented as "device" must be device memory of the GPU that
 *     was current when the context was created; "host" pointers are ordinary
 *     host memory;
 *   - the caller owns every buffer it passes; the library neither frees nor
 *     keeps caller pointers after a call returns; the context owns its own
 *     device workspace (about 4 n^2 + 8 n k complex numbers) and releases it
 *     in chfsi_release;
 *   - work is queued on the stream given at creation; calls return after
 *     their results are complete (they synchronize that stream);
 *   - errors are returned as chfsi_status; nothing is thrown or aborted;
 *     chfsi_last_error() gives a message for the last failure of a context;
 *     a failed call leaves the context usable;
 *   - a context is not thread-safe: one host thread at a time.
 */
#ifndef CHFSI_H
#define CHFSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chfsi_ctx_s* chfsi_ctx;

typedef enum {
  CHFSI_OK = 0,
  CHFSI_EINVAL = -1,  /* invalid argument (sizes, leading dimensions, null pointers, tol <= 0) */
  CHFSI_ENOTPD = -2,  /* S is not positive definite (column in chfsi_last_error) */
  CHFSI_ENOCONV = -3, /* max_iter reached; outputs hold the converged prefix (info.converged) */
  CHFSI_ENAN = -4,    /* non-finite value in the iteration (e.g. NaN in H) */
  CHFSI_ENOMEM = -5,  /* device allocation failed */
  CHFSI_EHIP = -6     /* HIP runtime error */
} chfsi_status;

typedef struct {
  int32_t degree;        /* Chebyshev filter degree m (default 20) */
  int32_t max_iter;      /* outer iterations before CHFSI_ENOCONV (default 1000) */
  int32_t lanczos_steps; /* Lanczos steps for the spectral bound (default 10, at most 96) */
  int32_t precision;     /* 0: FP64 throughout; 1: mixed - the Chebyshev filter in complex FP32
                            (FP32 matrix cores, FP32 accumulation) for the active columns after the
                            leading ones whose generalized residuals are below the switch (see
                            mixed_switch_digits), FP64 for those, for everything else and for the
                            final sweeps; accepted pairs meet the same FP64 tolerance;
                            2: every filter product in complex FP32 on the Ritz residual: the
                            recurrence of eq. (2) is linear, so with Y_0 the Ritz vectors of the last
                            Rayleigh-Ritz step (values mu, residual R = A Y_0 - Y_0 diag(mu) in FP64)
                            its iterates are Y_0 diag(t_i(mu)) + D_i, t_i the scalar recurrence (FP64)
                            and D_i the recurrence on R (FP32 products, errors relative to |D|, which
                            falls with the residual): no FP64 filter sweeps, the same FP64 tolerance;
                            the first iteration after a start block that is not a Ritz basis runs the
                            plain FP32 filter;
                            3: as 2 with the products' operands in FP16 (FP32 accumulation; A kept
                            as FP16 planes, each column of D scaled by a power of two to unit size),
                            errors relative to |D| at FP16's level; not accepted by
                            chfsi_batch_create */
  uint64_t seed;         /* Philox4x32-10 seed of the random start vectors (default 0) */
  int32_t profile;       /* 1: time the filter with device events (one pair around each filter call's degree steps) */
  int32_t qr_mode;       /* re-orthonormalization: 0 = CholeskyQR2, Householder when a Gram
                            matrix is not positive definite (default); 1 = Householder always */
  int32_t filter_tile;   /* filter kernel tile configuration (chfsi_zgemm's numbering; 0 = automatic) */
  int32_t filter_splitk; /* filter K split (0 = automatic, 1 = none, up to 16) */
  int32_t mixed_switch_digits; /* mixed precision: a column's filter turns FP64 once its generalized
                                  residual is below 10^-digits h_H (0 = default 6; 1 to 12); a switch
                                  below the FP32 filter's rounding floor costs iterations, not accuracy */
  int32_t reserved[3];
} chfsi_opts;

typedef struct {
  int32_t iterations;      /* outer iterations of Algorithm 1 */
  int32_t converged;       /* locked eigenpairs (>= nev on success) */
  int32_t warm_start;      /* 1 when the start block came from previous vectors */
  int32_t filter_launches; /* filter kernel launches (degree steps) */
  int32_t qr_householder;  /* re-orthonormalizations that used Householder QR */
  int32_t reserved_i;
  double filter_flops;     /* algorithmic filter work: sum over steps of 8 n^2 k_active */
  double filter_kernel_seconds; /* summed event-timed spans of the filter calls' launches (profile = 1, else 0) */
  double t_reduce, t_lanczos, t_filter, t_qr, t_rr, t_resid, t_total; /* seconds per phase */
  double b_upper;          /* Lanczos upper bound of the standard-form spectrum */
  double theta_min;        /* smallest Lanczos Ritz value */
  double h_H;              /* Lanczos estimate of ||H||_2 (lower bound); scale of the lock test */
  double a0, a;            /* filter scale point and lower end of the damped interval at exit */
  double max_rel_residual; /* max_j ||H x_j - lambda_j S x_j||_2 / h_H over returned pairs */
  int32_t iterations_fp32;      /* outer iterations whose filter ran in lower precision (FP32; FP16
                                   operands with precision 3) */
  int32_t filter_launches_fp32; /* of filter_launches, those in FP32 */
  double filter_flops_fp32;     /* of filter_flops, the FP32 part */
  double filter_kernel_seconds_fp32; /* of filter_kernel_seconds, the FP32 part */
} chfsi_info;

/* Fill *opts with the defaults listed above. */
void chfsi_default_opts(chfsi_opts* opts);

/* Human-readable name of a status code (static string). */
const char* chfsi_status_string(chfsi_status s);

/* Create a context for problems of size n on the current HIP device.
 * stream: a hipStream_t (0 = the null stream).  opts may be NULL (defaults).
 * CHFSI_EINVAL if n < 1 or an option is out of range. */
chfsi_status chfsi_create(chfsi_ctx* out, int64_t n, const chfsi_opts* opts, void* stream);

/* Free every device buffer owned by ctx.  NULL-safe. */
void chfsi_release(chfsi_ctx ctx);

/* Message of the last failed call on ctx ("" if none).  Owned by ctx.  With
 * ctx = NULL: the message of the calling thread's last failed
 * chfsi_zgemm_static call, or "null context" if there is none (owned by the
 * library, valid until that thread's next such call). */
const char* chfsi_last_error(chfsi_ctx ctx);

/* Forget the warm state kept from the previous solve (next solve starts cold). */
chfsi_status chfsi_reset(chfsi_ctx ctx);

/* Reduction to standard form (Section 3): S = L L^H (Cholesky) and
 * A = L^{-1} H L^{-H}, made exactly Hermitian.  H, S: device n x n.
 * S == NULL reuses the factor of the previous call (CHFSI_EINVAL if none).
 * The factors stay in ctx (chfsi_copy_factors reads them). */
chfsi_status chfsi_reduce(chfsi_ctx ctx, const void* H, int64_t ldh, const void* S, int64_t lds);

/* Solve H x = lambda S x for the nev smallest eigenpairs with a search block
 * of k = nev + nex vectors (Algorithm 1 with locking).  Sizes: 1 <= nev,
 * nev + nex <= n, and nex >= 1 unless nev = n (CHFSI_EINVAL otherwise): the
 * filter damps the interval that starts at the block's largest Ritz value,
 * which must not be a wanted one.
 *   H, S    device n x n; S == NULL reuses the cached factor of S (sequences
 *           with a fixed overlap matrix);
 *   V_warm  device n x kw approximate eigenvectors of the generalized problem
 *           (e.g. the previous solution), 0 <= kw <= k, may be NULL.  When
 *           NULL, the vectors and filter bounds kept from the previous solve
 *           on this context are used if their shape matches, else a seeded
 *           random block;
 *   tol     convergence: ||H x - lambda S x||_2 <= tol * h_H for each pair;
 *   evals   host, nev doubles, ascending;
 *   X       device n x nev, S-orthonormal eigenvectors (may be NULL);
 *   info    may be NULL.
 * CHFSI_ENOCONV leaves the converged prefix in evals/X (NaN beyond it). */
chfsi_status chfsi_solve(chfsi_ctx ctx, const void* H, int64_t ldh, const void* S, int64_t lds, int64_t nev, int64_t nex,
                         const void* V_warm, int64_t ldv, int64_t kw, double tol, double* evals, void* X, int64_t ldx,
                         chfsi_info* info);

/* ---- Step entry points ------------------------------------------------------
 * Each runs one step of Algorithm 1 on caller device buffers (n = the
 * context's size), on the context's stream, for testing and composition. */

/* Copy the factors of the last reduction: A (standard form), L (Cholesky
 * factor, zero upper triangle), Linv = L^{-1}.  Any pointer may be NULL. */
chfsi_status chfsi_copy_factors(chfsi_ctx ctx, void* A, int64_t lda, void* L, int64_t ldl, void* Linv, int64_t ldi);

/* Chebyshev filter (eq. (2), scaled and shifted): Y (device n x k) is
 * overwritten with p(A) Y, p(t) = C_m((t - c)/e) / C_m((a0 - c)/e),
 * c = (a + b)/2, e = (b - a)/2.  Requires b > a, m >= 1.  With the context's
 * precision 1, 2 or 3 the recurrence runs in complex FP32 (A and Y rounded
 * to FP32, the result widened back to FP64; Y carries no Ritz values here,
 * so 2 and 3 filter like 1: chfsi_filter_ritz is their filter). */
chfsi_status chfsi_filter(chfsi_ctx ctx, const void* A, int64_t lda, void* Y, int64_t ldy, int64_t k, int32_t m, double a,
                          double b, double a0);

/* The same filter as the solver's precision 2 and 3 compute it (eq. (2) split by
 * linearity): Y (device n x k) holds Ritz vectors of A with Ritz values mu
 * (host, k FP64 values) and AY = A Y (device n x k, FP64, leading dimension
 * lday).  Y is overwritten with p(A) Y = Y diag(t_m(mu)) + D_m, where t_i is
 * the filter's recurrence on the scalars mu_j (FP64) and D_i the recurrence
 * on the Ritz residual A Y - Y diag(mu) (D_0 = 0), each column scaled by a
 * power of two to unit size, its products in complex FP32 (A rounded to
 * FP32) or, when the context has precision 3, with FP16 operands and FP32
 * accumulation (A Hermitian: its FP16 copy takes row m as the conjugate of
 * column m).  Exact for any mu in exact arithmetic; the rounding errors are
 * relative to |D|, so they shrink as the residual does.  Requires b > a,
 * m >= 1, 1 <= k <= n. */
chfsi_status chfsi_filter_ritz(chfsi_ctx ctx, const void* A, int64_t lda, void* Y, int64_t ldy, const void* AY,
                               int64_t lday, const double* mu, int64_t k, int32_t m, double a, double b, double a0);

/* Householder QR: Y (device n x k, k <= n) is overwritten with the explicit
 * orthonormal factor Q; R has a real diagonal with the sign opposite to the
 * pivot's real part (LAPACK convention). */
chfsi_status chfsi_qr(chfsi_ctx ctx, void* Y, int64_t ldy, int64_t k);

/* The solver's re-orthonormalization (Algorithm 1): Y (device n x k) is
 * overwritten with an orthonormal basis of its span, by CholeskyQR2 or, when
 * a Gram matrix is not numerically positive definite (or opts.qr_mode = 1),
 * by Householder QR.  *used_householder (may be NULL) tells which. */
chfsi_status chfsi_orthonormalize(chfsi_ctx ctx, void* Y, int64_t ldy, int64_t k, int32_t* used_householder);

/* Hermitian eigensolver of the reduced problem (Algorithm 1's Rayleigh-Ritz
 * step; exact to working accuracy): G (device k x k, Hermitian, both
 * triangles read, read only) = Z diag(w) Z^H, w host (k, ascending), Z device
 * k x k.  Cyclic Jacobi (one workgroup up to k = 96, block-ordered sweeps
 * above), eigenvector refinement once G is nearly diagonal. */
chfsi_status chfsi_eigh(chfsi_ctx ctx, const void* G, int64_t ldg, int64_t k, double* w, void* Z, int64_t ldz);

/* Rayleigh-Ritz on an orthonormal block: G = Y^H A Y, G = Z diag(mu) Z^H,
 * Y <- Y Z.  Y device n x k, mu host k (ascending). */
chfsi_status chfsi_rayleigh_ritz(chfsi_ctx ctx, const void* A, int64_t lda, void* Y, int64_t ldy, int64_t k, double* mu);

/* Generalized residual norms rho_j = ||L (A y_j - mu_j y_j)||_2
 * (= ||H x_j - mu_j S x_j|| for x = L^{-H} y).  A, L, Y device; mu, rho host. */
chfsi_status chfsi_residuals(chfsi_ctx ctx, const void* A, int64_t lda, const void* L, int64_t ldl, const void* Y,
                             int64_t ldy, int64_t k, const double* mu, double* rho);

/* Lanczos with full re-orthogonalization on A (device n x n) from the random
 * vector of (seed, stream_id): out (host, 3) = {smallest Ritz value, largest
 * Ritz value, largest + ||last residual||} (the upper bound). */
chfsi_status chfsi_lanczos(chfsi_ctx ctx, const void* A, int64_t lda, int32_t steps, uint64_t seed, uint32_t stream_id,
                           double* out);

/* Random start block: Y(i, j) (device, n x k) = complex Gaussian number
 * i + (j + col0) n of Philox4x32-10 stream `stream_id` under `seed`
 * (counter (idx lo, idx hi, stream_id, 0), key (seed lo, seed hi); two 53-bit
 * uniforms, Box-Muller). */
chfsi_status chfsi_random_block(chfsi_ctx ctx, uint64_t seed, uint32_t stream_id, int64_t col0, void* Y, int64_t ldy,
                                int64_t k);

/* Raw Philox4x32-10 blocks: ctr (device, 4 count u32), key (device, 2 count),
 * out (device, 4 count). */
chfsi_status chfsi_philox(chfsi_ctx ctx, const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count);

/* The library's complex GEMM with its three-term epilogue:
 *   C = alpha op(A) op(B) + beta X + gamma Z,   op in {0: none, 1: conj-transpose}
 * op(A) M x K, op(B) K x N; X, Z may be NULL; C may alias X or Z.
 * flags bits 0-4: 1 op(A) lower-triangular, 2 op(A) upper, 4 op(B) lower,
 * 8 op(B) upper (zeros stored), 16 only tiles meeting the lower triangle of C;
 * bits 8-15: tile configuration (0 = automatic choice; 1 64x64x16, 2 32x32x16,
 * 3 64x64x8, 4 128x64x8, 5 64x128x8, 6 128x128x8, 7 64x32x16, 8 64x64x8 and
 * 9 64x32x16 with room for four workgroups per CU, 10 64x48x16, 11 64x64x16
 * with eight waves per workgroup, 12 64x80x16; 3-6, 8-10 and 12 only with
 * op = none on both sides); bits 16-23: K split (0 = automatic, 1 = none). */
chfsi_status chfsi_zgemm(chfsi_ctx ctx, int32_t opA, int32_t opB, int64_t M, int64_t N, int64_t K, double alpha,
                         const void* A, int64_t lda, const void* B, int64_t ldb, double beta, const void* X, int64_t ldx,
                         double gamma, const void* Z, int64_t ldz, void* C, int64_t ldc, int32_t flags);

/* Bytes of the fixed per-GPU scratch of chfsi_zgemm_static. */
#define CHFSI_STATIC_SCRATCH_BYTES ((int64_t)64 << 20)

/* Allocation-free chfsi_zgemm, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops and harnesses that forbid
 * hipMalloc): the same operation, arguments, flags and kernels as chfsi_zgemm,
 * without a context.  The work is queued on `stream` (a hipStream_t, NULL =
 * the null stream) and the call returns without waiting for it.  It calls no
 * hipMalloc / hipFree: the split-K partial tiles (split x M x N complex
 * numbers) live in a fixed device array of CHFSI_STATIC_SCRATCH_BYTES per GPU
 * that the library holds until the process ends.  An automatic split
 * (flags bits 16-23 = 0) is limited to what fits there; an explicit split
 * whose partial tiles exceed it returns CHFSI_EINVAL before any work is
 * queued.  Every call on one GPU uses that GPU's one array: calls whose work
 * overlaps in time on the same GPU (other streams, other host threads) race
 * and must be ordered by the caller.  Errors as chfsi_zgemm;
 * chfsi_last_error(NULL) gives the message of the calling thread's last
 * failed call of this function. */
chfsi_status chfsi_zgemm_static(void* stream, int32_t opA, int32_t opB, int64_t M, int64_t N, int64_t K,
                                double alpha, const void* A, int64_t lda, const void* B, int64_t ldb, double beta,
                                const void* X, int64_t ldx, double gamma, const void* Z, int64_t ldz, void* C,
                                int64_t ldc, int32_t flags);

/* ---- Batching -----------------------------------------------------------------
 * One solver per k-point for a fixed set of independent sequences (Section 2:
 * one sequence of eigenproblems per k-point, all of one SCF step solved
 * together).  A batch solve runs Algorithm 1 for every member in lockstep:
 * each outer iteration launches the degree steps of all members' Chebyshev
 * filters (eq. (2)) as one persistent grouped launch per step and precision,
 * then orthonormalizes, projects and locks each member on its own stream.
 * The grouped step's tile shape is chosen online: the first outer iterations
 * of each precision try the candidate shapes on the real work and the one
 * with the highest measured rate is kept for the rest of the batch's life
 * (the block-size study of Sec. 3 and Fig. 2, made automatic).  With use_graph = 1
 * the degree steps of an iteration replay as one captured HIP graph whose
 * kernels read the members' widths, pointers and alpha / beta / gamma
 * (eq. (2)) from device memory, so the same graph serves every iteration
 * while columns lock.  Each member keeps its block and bounds between calls
 * and warm-starts from them, as chfsi_solve does. */
typedef struct chfsi_batch_s* chfsi_batch;

typedef struct {
  int32_t tile_config;        /* grouped step tile configuration in use (FP64) */
  int32_t tile_config_fp32;   /* same for the FP32 steps (0: none ran yet) */
  int32_t graph;              /* 1 if the degree steps ran as captured graphs */
  int32_t outer_iterations;   /* lockstep iterations of this call */
  int32_t grouped_launches;   /* grouped step launches of this call */
  int32_t converged_members;  /* members that returned CHFSI_OK */
  double filter_flops;        /* algorithmic filter flops of this call, 8 n^2 k_a per member and step */
  double filter_seconds;      /* device time of the grouped steps (events around each iteration's steps) */
  double seconds;             /* wall time of the call */
  double tile_rate[16];       /* measured filter TFLOP/s per tile configuration (0: not tried; FP64) */
} chfsi_batch_report;

/* Create `count` (1..1024) member solvers of sizes n[0..count-1] on the
 * current device, each with the options *opts (NULL: defaults; filter_tile
 * != 0 pins the grouped tile shape instead of choosing it online; profile is
 * ignored).  Streams are created and owned by the batch.  CHFSI_EINVAL on bad
 * sizes or options. */
chfsi_status chfsi_batch_create(chfsi_batch* out, int32_t count, const int64_t* n, const chfsi_opts* opts,
                                int32_t use_graph);

/* Solve one problem per member: H[i], S[i] device n_i x n_i column-major
 * (S[i] NULL keeps member i's previous factor, as in chfsi_solve); nev[i],
 * nex[i] as in chfsi_solve; evals[i] host, nev[i] doubles; X[i] device
 * n_i x nev[i] or NULL.  infos (count entries) and statuses (count entries)
 * receive each member's chfsi_info and status; report (may be NULL) the
 * batch-level figures.  Returns CHFSI_OK when every member converged, else
 * the first failing member's status; argument errors return CHFSI_EINVAL
 * before any device work.  Input buffers must be ready on the device (the
 * call synchronizes the device before starting); outputs are complete on
 * return. */
chfsi_status chfsi_batch_solve(chfsi_batch b, const void* const* H, const int64_t* ldh, const void* const* S,
                               const int64_t* lds, const int64_t* nev, const int64_t* nex, double tol,
                               double* const* evals, void* const* X, const int64_t* ldx, chfsi_info* infos,
                               int32_t* statuses, chfsi_batch_report* report);

/* Forget every member's warm state (the next solve starts cold). */
chfsi_status chfsi_batch_reset(chfsi_batch b);

/* Message of the last error (first failing member's, for a solve). */
const char* chfsi_batch_last_error(chfsi_batch b);

/* Free the members, streams and graphs.  NULL-safe. */
void chfsi_batch_release(chfsi_batch b);

/* ---- Serving ------------------------------------------------------------------
 * A request loop over many sequences of problems (one sequence per k-point,
 * Section 2).  Worker threads each own a HIP stream and a solver context, so
 * admitted requests run concurrently on the device.  Each sequence keeps its
 * last block of k vectors (generalized space) and its filter bounds in device
 * memory and warm-starts its next problem from them.  A request is admitted
 * when the device memory it needs (a solver context for its size plus its
 * sequence's state) fits the budget; idle workers' contexts are released to
 * make room.  Problems of one sequence run in submission order, one at a time.
 * Results do not depend on what else runs: every solve uses its own context,
 * stream and deterministic kernels. */
typedef struct chfsi_server_s* chfsi_server;

typedef struct {
  int32_t workers;          /* concurrent solves (1..64) */
  int32_t reserved;
  int64_t hbm_budget_bytes; /* device memory for contexts + resident sequence state */
  chfsi_opts opts;          /* solver options of every request */
} chfsi_server_config;

typedef struct {
  int64_t submitted, completed, failed, queued, running;
  int64_t bytes_in_use, peak_bytes, budget_bytes;
  double solves_per_second; /* completed / (last completion - first submission) */
  double p50_latency, p99_latency, mean_latency; /* seconds, submission to completion */
} chfsi_server_statistics;

/* Start a server on the current HIP device.  CHFSI_EINVAL on bad config. */
chfsi_status chfsi_server_create(chfsi_server* out, const chfsi_server_config* cfg);

/* Queue one problem of sequence `seq`.  H, S: device n x n; evals: host,
 * nev doubles; X: device n x nev (may be NULL).  All four must stay valid
 * until chfsi_server_wait returns for the ticket.  S == NULL: the overlap
 * matrix is the one of the sequence's last request that passed S (same n),
 * which must then still be valid and unchanged until this request
 * completes; the request reuses that matrix's Cholesky factor when a
 * worker's context still holds it (such requests go to that worker when it
 * is idle), else factors it again (CHFSI_EINVAL at completion if the
 * sequence never passed S).  The problem is solved as by chfsi_solve,
 * warm-started from the sequence's previous problem when its size and block
 * width match.  A worker's context serves every problem size up to the
 * largest it has taken; a larger one grows it, or replaces it when the
 * budget does not allow growth. */
chfsi_status chfsi_server_submit(chfsi_server s, int64_t seq, int64_t n, const void* H, int64_t ldh, const void* S,
                                 int64_t lds, int64_t nev, int64_t nex, double tol, double* evals, void* X, int64_t ldx,
                                 int64_t* ticket);

/* Block until the ticket's request has finished; returns its status
 * (CHFSI_ENOMEM when it can never fit the budget).  The ticket is consumed. */
chfsi_status chfsi_server_wait(chfsi_server s, int64_t ticket, chfsi_info* info, double* latency_seconds);

/* Throughput, latency percentiles and memory of the requests so far. */
chfsi_status chfsi_server_stats(chfsi_server s, chfsi_server_statistics* out);

/* Drop a sequence's resident state (CHFSI_EINVAL while it has work queued). */
chfsi_status chfsi_server_release_sequence(chfsi_server s, int64_t seq);

/* Message of the last failed request. */
const char* chfsi_server_last_error(chfsi_server s);

/* Finish running requests, fail queued ones, free everything.  NULL-safe. */
void chfsi_server_destroy(chfsi_server s);

#ifdef __cplusplus
}
#endif

#endif /* CHFSI_H */
