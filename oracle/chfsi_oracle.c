/*
 * Plain CPU oracle for the Chebyshev-filtered subspace iteration (ChFSI) of
 * Berljafa & Di Napoli, "A Parallel and Scalable Iterative Solver for
 * Sequences of Dense Eigenproblems Arising in FLAPW" (arXiv 1305.5120).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the
 * product path never does.  It shares no code, header or table with the
 * GPU library.
 *
 * Conventions
 *   - complex128 numbers are (re, im) pairs of doubles; every complex
 *     product is written out as (ac - bd, ad + bc) so that no libgcc helper,
 *     FMA contraction or fast-math rewrite changes the rounding;
 *   - matrices are column-major with an explicit leading dimension;
 *   - no BLAS or LAPACK; OpenMP (if enabled) only splits independent output
 *     columns, so the summation order of every element is the one written.
 *
 * Parity status of each function is stated in its comment.  Every function
 * below is pinned by the CPU test suite against something other than itself
 * (closed forms, constructed factors, brute force, library routines used as
 * independent checks); the iteration trajectory of the full solve (iteration
 * counts, intermediate blocks, the exact value of the Lanczos bound) is not
 * fixed by the paper and is compared only through invariants.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cplx;

/* Thread count of the OpenMP loops (timing on a chosen number of cores);
   returns the count in effect before the call, 1 without OpenMP.  n < 1
   leaves it unchanged. */
int orc_set_threads(int n) {
#ifdef _OPENMP
  int prev = omp_get_max_threads();
  if (n >= 1) omp_set_num_threads(n);
  return prev;
#else
  (void)n;
  return 1;
#endif
}

static inline cplx c_mul(cplx a, cplx b) { cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
/* conj(a) * b */
static inline cplx c_cmul(cplx a, cplx b) { cplx r = {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; return r; }
static inline cplx c_add(cplx a, cplx b) { cplx r = {a.re + b.re, a.im + b.im}; return r; }
static inline cplx c_sub(cplx a, cplx b) { cplx r = {a.re - b.re, a.im - b.im}; return r; }
static inline cplx c_scale(double s, cplx a) { cplx r = {s * a.re, s * a.im}; return r; }
static inline cplx c_conj(cplx a) { cplx r = {a.re, -a.im}; return r; }
static inline double c_abs2(cplx a) { return a.re * a.re + a.im * a.im; }
static inline cplx c_div(cplx a, cplx b) {
  /* straightforward quotient a * conj(b) / |b|^2; the operands seen here are
     far from overflow */
  double d = c_abs2(b);
  cplx r = {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
  return r;
}

#define AT(M, ld, i, j) ((M)[(size_t)(i) + (size_t)(j) * (size_t)(ld)])

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,        */
/* "Parallel random numbers: as easy as 1, 2, 3", SC 2011).  Used for the    */
/* random start block and the Lanczos start vectors, which the method draws. */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    uint64_t p0 = (uint64_t)0xD2511F53u * x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/*
 * Complex Gaussian entry number e of stream s under seed:
 *   counter = (e mod 2^32, e div 2^32, s, 0), key = (seed mod 2^32, seed div 2^32);
 *   u1 = ((w0 << 32 | w1) >> 11 + 1/2) 2^-53, u2 likewise from (w2, w3);
 *   z  = sqrt(-2 ln u1) (cos 2 pi u2 + i sin 2 pi u2)   (Box-Muller).
 * Real and imaginary parts are independent N(0,1).
 */
static cplx gauss_entry(uint64_t seed, uint32_t stream, uint64_t e) {
  uint32_t ctr[4] = {(uint32_t)e, (uint32_t)(e >> 32), stream, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  uint64_t q1 = (((uint64_t)w[0] << 32) | w[1]) >> 11;
  uint64_t q2 = (((uint64_t)w[2] << 32) | w[3]) >> 11;
  double u1 = ((double)q1 + 0.5) * 0x1p-53;
  double u2 = ((double)q2 + 0.5) * 0x1p-53;
  double r = sqrt(-2.0 * log(u1));
  double t = 6.283185307179586476925286766559 * u2;
  cplx z = {r * cos(t), r * sin(t)};
  return z;
}

/* n x k block, entry (i, j) is entry number i + j*n of the stream. */
void orc_gauss_block(uint64_t seed, uint32_t stream, int64_t n, int64_t k, int64_t col0, cplx* Y, int64_t ldy) {
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < n; i++)
      AT(Y, ldy, i, j) = gauss_entry(seed, stream, (uint64_t)i + (uint64_t)(j + col0) * (uint64_t)n);
}

/* ------------------------------------------------------------------------ */
/* Dense building blocks                                                     */
/* ------------------------------------------------------------------------ */

/* C(:, j) = A * B(:, j) for j < k;  A is n x n. */
static void matmul(int64_t n, int64_t k, const cplx* A, int64_t lda, const cplx* B, int64_t ldb, cplx* C, int64_t ldc) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < k; j++) {
    cplx* c = &AT(C, ldc, 0, j);
    for (int64_t i = 0; i < n; i++) { c[i].re = 0.0; c[i].im = 0.0; }
    for (int64_t p = 0; p < n; p++) {
      cplx b = AT(B, ldb, p, j);
      const cplx* a = &AT(A, lda, 0, p);
      for (int64_t i = 0; i < n; i++) c[i] = c_add(c[i], c_mul(a[i], b));
    }
  }
}

/* 2-norm of a complex vector, plain sum of squares. */
static double vnorm(int64_t n, const cplx* x) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) s += c_abs2(x[i]);
  return sqrt(s);
}

/* x^H y */
static cplx vdot(int64_t n, const cplx* x, const cplx* y) {
  cplx s = {0.0, 0.0};
  for (int64_t i = 0; i < n; i++) s = c_add(s, c_cmul(x[i], y[i]));
  return s;
}

/* ------------------------------------------------------------------------ */
/* Reduction to standard form (Section 3, text after Algorithm 1): the      */
/* overlap matrix is factored as S = L L^H and the Hamiltonian becomes       */
/* A = L^{-1} H L^{-H}.  The paper writes transposes; for complex Hermitian  */
/* input they are conjugate transposes.                                      */
/* ------------------------------------------------------------------------ */

/* Unblocked Cholesky S = L L^H, L lower with a real positive diagonal; the
   strict upper triangle of L is set to zero.  Returns 0, or j+1 when the
   pivot of column j is not positive (S not positive definite). */
int64_t orc_cholesky(int64_t n, const cplx* S, int64_t lds, cplx* L, int64_t ldl) {
  for (int64_t j = 0; j < n; j++)
    for (int64_t i = 0; i < n; i++) {
      if (i >= j) AT(L, ldl, i, j) = AT(S, lds, i, j);
      else { AT(L, ldl, i, j).re = 0.0; AT(L, ldl, i, j).im = 0.0; }
    }
  for (int64_t j = 0; j < n; j++) {
    double d = AT(L, ldl, j, j).re;
    for (int64_t p = 0; p < j; p++) d -= c_abs2(AT(L, ldl, j, p));
    if (!(d > 0.0)) return j + 1;
    double ljj = sqrt(d);
    AT(L, ldl, j, j).re = ljj;
    AT(L, ldl, j, j).im = 0.0;
    for (int64_t i = j + 1; i < n; i++) {
      cplx s = AT(L, ldl, i, j);
      /* s -= sum_p L(i,p) conj(L(j,p)) */
      for (int64_t p = 0; p < j; p++) s = c_sub(s, c_mul(AT(L, ldl, i, p), c_conj(AT(L, ldl, j, p))));
      AT(L, ldl, i, j) = c_scale(1.0 / ljj, s);
    }
  }
  return 0;
}

/* Solve L X = B in place by forward substitution for k right-hand sides. */
static void lower_solve(int64_t n, int64_t k, const cplx* L, int64_t ldl, cplx* B, int64_t ldb) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < k; j++) {
    cplx* b = &AT(B, ldb, 0, j);
    for (int64_t i = 0; i < n; i++) {
      cplx s = b[i];
      for (int64_t p = 0; p < i; p++) s = c_sub(s, c_mul(AT(L, ldl, i, p), b[p]));
      b[i] = c_scale(1.0 / AT(L, ldl, i, i).re, s);
    }
  }
}

/* Solve L^H X = B in place by back substitution for k right-hand sides. */
static void lower_h_solve(int64_t n, int64_t k, const cplx* L, int64_t ldl, cplx* B, int64_t ldb) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < k; j++) {
    cplx* b = &AT(B, ldb, 0, j);
    for (int64_t i = n - 1; i >= 0; i--) {
      cplx s = b[i];
      /* (L^H)(i,p) = conj(L(p,i)) for p > i */
      for (int64_t p = i + 1; p < n; p++) s = c_sub(s, c_cmul(AT(L, ldl, p, i), b[p]));
      b[i] = c_scale(1.0 / AT(L, ldl, i, i).re, s);
    }
  }
}

/* A = L^{-1} H L^{-H}: W = L^{-1} H, then A = L^{-1} W^H (equal because H is
   Hermitian), then A <- (A + A^H)/2. */
void orc_reduce(int64_t n, const cplx* H, int64_t ldh, const cplx* L, int64_t ldl, cplx* A, int64_t lda) {
  cplx* W = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)n);
  for (int64_t j = 0; j < n; j++)
    for (int64_t i = 0; i < n; i++) AT(W, n, i, j) = AT(H, ldh, i, j);
  lower_solve(n, n, L, ldl, W, n);
  for (int64_t j = 0; j < n; j++)
    for (int64_t i = 0; i < n; i++) AT(A, lda, i, j) = c_conj(AT(W, n, j, i));
  lower_solve(n, n, L, ldl, A, lda);
  for (int64_t j = 0; j < n; j++) {
    for (int64_t i = j + 1; i < n; i++) {
      cplx x = AT(A, lda, i, j), y = c_conj(AT(A, lda, j, i));
      cplx m = c_scale(0.5, c_add(x, y));
      AT(A, lda, i, j) = m;
      AT(A, lda, j, i) = c_conj(m);
    }
    AT(A, lda, j, j).im = 0.0;
  }
  free(W);
}

/* X = L^{-H} Y (back-transform of standard-form vectors to the generalized
   eigenvectors), in place on Y (n x k). */
void orc_backtransform(int64_t n, int64_t k, const cplx* L, int64_t ldl, cplx* Y, int64_t ldy) {
  lower_h_solve(n, k, L, ldl, Y, ldy);
}

/* Y = L^H V (generalized-space vectors mapped to the standard form). */
void orc_lh_times(int64_t n, int64_t k, const cplx* L, int64_t ldl, const cplx* V, int64_t ldv, cplx* Y, int64_t ldy) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < n; i++) {
      cplx s = {0.0, 0.0};
      for (int64_t p = i; p < n; p++) s = c_add(s, c_cmul(AT(L, ldl, p, i), AT(V, ldv, p, j)));
      AT(Y, ldy, i, j) = s;
    }
}

/* Y = L R, L lower triangular. */
static void lower_times(int64_t n, int64_t k, const cplx* L, int64_t ldl, const cplx* R, int64_t ldr, cplx* Y, int64_t ldy) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < n; i++) {
      cplx s = {0.0, 0.0};
      for (int64_t p = 0; p <= i; p++) s = c_add(s, c_mul(AT(L, ldl, i, p), AT(R, ldr, p, j)));
      AT(Y, ldy, i, j) = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Cyclic Jacobi for a Hermitian matrix (the small Rayleigh-Ritz problem of  */
/* Algorithm 1; the paper uses MRRR there, any exact Hermitian eigensolver   */
/* gives the same result).                                                   */
/* ------------------------------------------------------------------------ */

/* Eigen-decomposition G = Z diag(w) Z^H of a Hermitian k x k matrix by
   row-cyclic Jacobi with complex rotations.  G is destroyed.  Eigenvalues
   come back ascending (ties keep their index order) with Z's columns in the
   same order.  Returns the number of sweeps. */
int orc_jacobi_eigh(int64_t k, cplx* G, int64_t ldg, double* w, cplx* Z, int64_t ldz) {
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < k; i++) { AT(Z, ldz, i, j).re = (i == j) ? 1.0 : 0.0; AT(Z, ldz, i, j).im = 0.0; }
  for (int64_t i = 0; i < k; i++) AT(G, ldg, i, i).im = 0.0;
  double fro2 = 0.0;
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < k; i++) fro2 += c_abs2(AT(G, ldg, i, j));
  const double skip2 = 1e-36 * fro2; /* |g|^2 below this is already zero to working accuracy */
  int sweeps = 0;
  for (; sweeps < 100; sweeps++) {
    double off2 = 0.0;
    for (int64_t j = 0; j < k; j++)
      for (int64_t i = 0; i < k; i++)
        if (i != j) off2 += c_abs2(AT(G, ldg, i, j));
    if (off2 <= 1e-32 * fro2 || off2 == 0.0) break;
    int rotated = 0;
    for (int64_t p = 0; p < k - 1; p++) {
      for (int64_t q = p + 1; q < k; q++) {
        cplx g = AT(G, ldg, p, q);
        double ag2 = c_abs2(g);
        if (ag2 <= skip2 || ag2 == 0.0) continue;
        rotated = 1;
        double ag = sqrt(ag2);
        cplx u = {g.re / ag, g.im / ag}; /* g = |g| u */
        double app = AT(G, ldg, p, p).re, aqq = AT(G, ldg, q, q).re;
        /* real symmetric 2x2 [[app, ag], [ag, aqq]]: rotation [[c, s], [-s, c]] */
        double tau = (aqq - app) / (2.0 * ag);
        double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        double c = 1.0 / sqrt(1.0 + t * t);
        double s = t * c;
        /* J = [[u c, u s], [-s, c]] acting on columns p, q */
        cplx j00 = c_scale(c, u), j01 = c_scale(s, u);
        double j10 = -s, j11 = c;
        for (int64_t i = 0; i < k; i++) {
          cplx gp = AT(G, ldg, i, p), gq = AT(G, ldg, i, q);
          AT(G, ldg, i, p) = c_add(c_mul(gp, j00), c_scale(j10, gq));
          AT(G, ldg, i, q) = c_add(c_mul(gp, j01), c_scale(j11, gq));
        }
        for (int64_t i = 0; i < k; i++) {
          cplx gp = AT(G, ldg, p, i), gq = AT(G, ldg, q, i);
          AT(G, ldg, p, i) = c_add(c_cmul(j00, gp), c_scale(j10, gq));
          AT(G, ldg, q, i) = c_add(c_cmul(j01, gp), c_scale(j11, gq));
        }
        AT(G, ldg, p, q).re = 0.0; AT(G, ldg, p, q).im = 0.0;
        AT(G, ldg, q, p).re = 0.0; AT(G, ldg, q, p).im = 0.0;
        AT(G, ldg, p, p).re = app - t * ag; AT(G, ldg, p, p).im = 0.0;
        AT(G, ldg, q, q).re = aqq + t * ag; AT(G, ldg, q, q).im = 0.0;
        for (int64_t i = 0; i < k; i++) {
          cplx zp = AT(Z, ldz, i, p), zq = AT(Z, ldz, i, q);
          AT(Z, ldz, i, p) = c_add(c_mul(zp, j00), c_scale(j10, zq));
          AT(Z, ldz, i, q) = c_add(c_mul(zp, j01), c_scale(j11, zq));
        }
      }
    }
    if (!rotated) break;
  }
  /* stable ascending order */
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
  for (int64_t i = 0; i < k; i++) idx[i] = i;
  for (int64_t i = 1; i < k; i++) {
    int64_t v = idx[i];
    double key = AT(G, ldg, v, v).re;
    int64_t j = i - 1;
    while (j >= 0 && AT(G, ldg, idx[j], idx[j]).re > key) { idx[j + 1] = idx[j]; j--; }
    idx[j + 1] = v;
  }
  cplx* Zs = (cplx*)malloc(sizeof(cplx) * (size_t)k * (size_t)(k > 0 ? k : 1));
  for (int64_t j = 0; j < k; j++) {
    w[j] = AT(G, ldg, idx[j], idx[j]).re;
    for (int64_t i = 0; i < k; i++) Zs[i + j * k] = AT(Z, ldz, i, idx[j]);
  }
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < k; i++) AT(Z, ldz, i, j) = Zs[i + j * k];
  free(Zs);
  free(idx);
  return sweeps;
}

/* ------------------------------------------------------------------------ */
/* Householder QR (Algorithm 1, re-orthonormalization step).                 */
/* Reflector H = I - tau v v^H with v(0) = 1 and H^H x = beta e_1, beta real */
/* with the sign opposite to Re x(0); Q = H_0 H_1 ... H_{k-1} [I_k; 0].      */
/* ------------------------------------------------------------------------ */
void orc_householder_qr(int64_t n, int64_t k, cplx* Y, int64_t ldy, cplx* Q, int64_t ldq, cplx* R, int64_t ldr) {
  cplx* tau = (cplx*)malloc(sizeof(cplx) * (size_t)(k > 0 ? k : 1));
  for (int64_t j = 0; j < k; j++) {
    cplx alpha = AT(Y, ldy, j, j);
    double xnorm = vnorm(n - j - 1, &AT(Y, ldy, j + 1, j));
    if (xnorm == 0.0 && alpha.im == 0.0) {
      tau[j].re = 0.0; tau[j].im = 0.0;
      continue; /* H = I, R(j,j) = alpha */
    }
    double nrm = sqrt(c_abs2(alpha) + xnorm * xnorm);
    double beta = (alpha.re >= 0.0) ? -nrm : nrm;
    tau[j].re = (beta - alpha.re) / beta;
    tau[j].im = -alpha.im / beta;
    cplx denom = {alpha.re - beta, alpha.im};
    cplx one = {1.0, 0.0};
    cplx scal = c_div(one, denom);
    for (int64_t i = j + 1; i < n; i++) AT(Y, ldy, i, j) = c_mul(AT(Y, ldy, i, j), scal);
    AT(Y, ldy, j, j).re = beta; AT(Y, ldy, j, j).im = 0.0;
    /* apply H^H = I - conj(tau) v v^H to the trailing columns */
    cplx ctau = c_conj(tau[j]);
#pragma omp parallel for schedule(static)
    for (int64_t c = j + 1; c < k; c++) {
      cplx* y = &AT(Y, ldy, 0, c);
      cplx wsum = y[j]; /* v(j) = 1 */
      for (int64_t i = j + 1; i < n; i++) wsum = c_add(wsum, c_cmul(AT(Y, ldy, i, j), y[i]));
      cplx f = c_mul(ctau, wsum);
      y[j] = c_sub(y[j], f);
      for (int64_t i = j + 1; i < n; i++) y[i] = c_sub(y[i], c_mul(AT(Y, ldy, i, j), f));
    }
  }
  if (R) {
    for (int64_t j = 0; j < k; j++)
      for (int64_t i = 0; i < k; i++) {
        if (i <= j) AT(R, ldr, i, j) = AT(Y, ldy, i, j);
        else { AT(R, ldr, i, j).re = 0.0; AT(R, ldr, i, j).im = 0.0; }
      }
  }
  /* Q = H_0 ... H_{k-1} applied to the first k columns of the identity */
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < n; i++) { AT(Q, ldq, i, j).re = (i == j) ? 1.0 : 0.0; AT(Q, ldq, i, j).im = 0.0; }
  for (int64_t j = k - 1; j >= 0; j--) {
    cplx t = tau[j];
    if (t.re == 0.0 && t.im == 0.0) continue;
#pragma omp parallel for schedule(static)
    for (int64_t c = j; c < k; c++) {
      cplx* q = &AT(Q, ldq, 0, c);
      cplx wsum = q[j];
      for (int64_t i = j + 1; i < n; i++) wsum = c_add(wsum, c_cmul(AT(Y, ldy, i, j), q[i]));
      cplx f = c_mul(t, wsum);
      q[j] = c_sub(q[j], f);
      for (int64_t i = j + 1; i < n; i++) q[i] = c_sub(q[i], c_mul(AT(Y, ldy, i, j), f));
    }
  }
  free(tau);
}

/* ------------------------------------------------------------------------ */
/* Lanczos estimate of the spectrum's ends (Algorithm 1, first step; the     */
/* upper bound follows Zhou & Li: largest Ritz value plus the norm of the    */
/* last residual vector).  Full re-orthogonalization, steps = min(steps, n). */
/* out[0] = smallest Ritz value, out[1] = largest Ritz value,                */
/* out[2] = upper bound b = out[1] + ||f_steps||.                            */
/* ------------------------------------------------------------------------ */
void orc_lanczos(int64_t n, const cplx* A, int64_t lda, int64_t steps, const cplx* v0, double* out) {
  if (steps > n) steps = n;
  cplx* V = (cplx*)calloc((size_t)n * (size_t)(steps + 1), sizeof(cplx));
  cplx* w = (cplx*)malloc(sizeof(cplx) * (size_t)n);
  double* alpha = (double*)calloc((size_t)steps + 1, sizeof(double));
  double* beta = (double*)calloc((size_t)steps + 2, sizeof(double));
  double nv = vnorm(n, v0);
  for (int64_t i = 0; i < n; i++) V[i] = c_scale(1.0 / nv, v0[i]);
  int64_t used = 0;
  double fnorm = 0.0;
  for (int64_t j = 0; j < steps; j++) {
    matmul(n, 1, A, lda, &V[(size_t)j * n], n, w, n);
    alpha[j] = vdot(n, &V[(size_t)j * n], w).re;
    for (int64_t i = 0; i < n; i++) {
      w[i] = c_sub(w[i], c_scale(alpha[j], V[(size_t)j * n + i]));
      if (j > 0) w[i] = c_sub(w[i], c_scale(beta[j], V[(size_t)(j - 1) * n + i]));
    }
    /* full re-orthogonalization, two passes */
    for (int pass = 0; pass < 2; pass++)
      for (int64_t p = 0; p <= j; p++) {
        cplx h = vdot(n, &V[(size_t)p * n], w);
        for (int64_t i = 0; i < n; i++) w[i] = c_sub(w[i], c_mul(V[(size_t)p * n + i], h));
      }
    used = j + 1;
    fnorm = vnorm(n, w);
    beta[j + 1] = fnorm;
    if (j + 1 < steps) {
      if (!(fnorm > 0.0)) break; /* invariant subspace found: Ritz values are exact */
      for (int64_t i = 0; i < n; i++) V[(size_t)(j + 1) * n + i] = c_scale(1.0 / fnorm, w[i]);
    }
  }
  /* eigenvalues of the real symmetric tridiagonal T (used x used) */
  cplx* T = (cplx*)calloc((size_t)used * (size_t)used, sizeof(cplx));
  cplx* Z = (cplx*)calloc((size_t)used * (size_t)used, sizeof(cplx));
  double* th = (double*)malloc(sizeof(double) * (size_t)used);
  for (int64_t i = 0; i < used; i++) {
    T[i + i * used].re = alpha[i];
    if (i + 1 < used) {
      T[(i + 1) + i * used].re = beta[i + 1];
      T[i + (i + 1) * used].re = beta[i + 1];
    }
  }
  orc_jacobi_eigh(used, T, used, th, Z, used);
  out[0] = th[0];
  out[1] = th[used - 1];
  out[2] = th[used - 1] + fnorm;
  free(T); free(Z); free(th); free(V); free(w); free(alpha); free(beta);
}

/* ------------------------------------------------------------------------ */
/* Chebyshev filter (Algorithm 1, filter step; three-term recurrence of      */
/* Chebyshev polynomials of the first kind, eq. (2)).  The recurrence is     */
/* applied to (A - c I)/e, which maps the unwanted interval [a, b] onto      */
/* [-1, 1], and is scaled so that the polynomial equals 1 at a0:             */
/*   e = (b - a)/2, c = (b + a)/2, sigma_1 = e/(a0 - c), tau = 2/sigma_1,     */
/*   Y_1 = (sigma_1/e)(A - cI) Y_0,                                          */
/*   Y_i = (2 sigma_i/e)(A - cI) Y_{i-1} - sigma_{i-1} sigma_i Y_{i-2},       */
/*   sigma_i = 1/(tau - sigma_{i-1}),                                        */
/* so that Y_m = p(A) Y_0 with p(t) = C_m((t - c)/e) / C_m((a0 - c)/e).       */
/* Y (n x k) is overwritten with Y_m.                                        */
/* ------------------------------------------------------------------------ */
void orc_filter(int64_t n, const cplx* A, int64_t lda, cplx* Y, int64_t ldy, int64_t k, int32_t m, double a, double b, double a0) {
  if (m < 1 || k < 1) return;
  double e = (b - a) / 2.0, c = (b + a) / 2.0;
  double sigma1 = e / (a0 - c);
  double tau = 2.0 / sigma1;
  cplx* prev = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)k); /* Y_{i-2} */
  cplx* cur = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)k);  /* Y_{i-1} */
  cplx* AY = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)k);
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < n; i++) prev[i + j * n] = AT(Y, ldy, i, j);
  /* step 1 */
  matmul(n, k, A, lda, prev, n, AY, n);
  double al = sigma1 / e;
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < n; i++) {
      size_t t = (size_t)i + (size_t)j * n;
      cur[t] = c_scale(al, c_sub(AY[t], c_scale(c, prev[t])));
    }
  double sigma = sigma1;
  for (int32_t s = 2; s <= m; s++) {
    double sn = 1.0 / (tau - sigma);
    matmul(n, k, A, lda, cur, n, AY, n);
    double a2 = 2.0 * sn / e, g = sigma * sn;
    for (int64_t j = 0; j < k; j++)
      for (int64_t i = 0; i < n; i++) {
        size_t t = (size_t)i + (size_t)j * n;
        cplx nv = c_sub(c_scale(a2, c_sub(AY[t], c_scale(c, cur[t]))), c_scale(g, prev[t]));
        prev[t] = cur[t];
        cur[t] = nv;
      }
    sigma = sn;
  }
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < n; i++) AT(Y, ldy, i, j) = cur[i + j * n];
  free(prev); free(cur); free(AY);
}

/* ------------------------------------------------------------------------ */
/* Rayleigh-Ritz (Algorithm 1): G = Y^H A Y (Hermitian part), G = Z diag(mu)  */
/* Z^H, Y <- Y Z.  mu ascending.                                             */
/* ------------------------------------------------------------------------ */
void orc_rayleigh_ritz(int64_t n, const cplx* A, int64_t lda, cplx* Y, int64_t ldy, int64_t k, double* mu) {
  cplx* W = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)k);
  cplx* G = (cplx*)malloc(sizeof(cplx) * (size_t)k * (size_t)k);
  cplx* Z = (cplx*)malloc(sizeof(cplx) * (size_t)k * (size_t)k);
  cplx* T = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)k);
  matmul(n, k, A, lda, Y, ldy, W, n);
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < k; i++) G[i + j * k] = vdot(n, &AT(Y, ldy, 0, i), &W[(size_t)j * n]);
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = j; i < k; i++) {
      cplx m = c_scale(0.5, c_add(G[i + j * k], c_conj(G[j + i * k])));
      G[i + j * k] = m;
      G[j + i * k] = c_conj(m);
    }
  orc_jacobi_eigh(k, G, k, mu, Z, k);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < n; i++) {
      cplx s = {0.0, 0.0};
      for (int64_t p = 0; p < k; p++) s = c_add(s, c_mul(AT(Y, ldy, i, p), Z[p + j * k]));
      T[(size_t)i + (size_t)j * n] = s;
    }
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < n; i++) AT(Y, ldy, i, j) = T[(size_t)i + (size_t)j * n];
  free(W); free(G); free(Z); free(T);
}

/* ------------------------------------------------------------------------ */
/* Residual norms of the generalized problem: for standard-form Ritz pairs   */
/* (mu_j, y_j), rho_j = || L (A y_j - mu_j y_j) ||_2, which equals            */
/* || H x_j - mu_j S x_j ||_2 for x_j = L^{-H} y_j.                           */
/* ------------------------------------------------------------------------ */
void orc_residuals(int64_t n, const cplx* A, int64_t lda, const cplx* L, int64_t ldl, const cplx* Y, int64_t ldy, int64_t k,
                   const double* mu, double* rho) {
  cplx* R = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)k);
  cplx* LR = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)k);
  matmul(n, k, A, lda, Y, ldy, R, n);
  for (int64_t j = 0; j < k; j++)
    for (int64_t i = 0; i < n; i++) R[(size_t)i + (size_t)j * n] = c_sub(R[(size_t)i + (size_t)j * n], c_scale(mu[j], AT(Y, ldy, i, j)));
  lower_times(n, k, L, ldl, R, n, LR, n);
  for (int64_t j = 0; j < k; j++) rho[j] = vnorm(n, &LR[(size_t)j * n]);
  free(R); free(LR);
}

/* ------------------------------------------------------------------------ */
/* Full solve: Algorithm 1 with locking, on the pencil (H, S).               */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t degree;        /* m */
  int32_t max_iter;
  int32_t lanczos_steps; /* k_L */
  int32_t have_bounds;   /* warm bounds given in bounds_in */
  uint64_t seed;
} orc_opts;

typedef struct {
  int32_t iterations;
  int32_t converged;
  int32_t status; /* 0 ok, -2 S not PD (column in info.bad_column), -3 not converged */
  int32_t bad_column;
  double b_upper, theta_min, h_H;
  double a0, a;      /* filter bounds at exit (warm state) */
  double filter_flops;
  double max_rel_residual;
} orc_info;

/*
 * Inputs: H, S (n x n Hermitian; S positive definite).  V_warm (n x kw, may
 * be NULL) are approximate generalized eigenvectors from the previous
 * problem of the sequence; missing columns are filled from the seeded random
 * stream 3.  bounds_in = {a0, a} from the previous solve when have_bounds.
 * Outputs: evals (nev, ascending), X (n x nev) generalized eigenvectors,
 * Y_state (n x k, may be NULL): the final standard-form block, the warm
 * state of the next solve.
 */
int32_t orc_solve(int64_t n, const cplx* H, int64_t ldh, const cplx* S, int64_t lds, int64_t nev, int64_t nex,
                  const cplx* V_warm, int64_t ldv, int64_t kw, const double* bounds_in, double tol, const orc_opts* opt,
                  double* evals, cplx* X, int64_t ldx, cplx* Y_state, orc_info* info) {
  memset(info, 0, sizeof(*info));
  int64_t k = nev + nex;
  /* sizes: at least one extra column unless the block is the whole space
     (the damped interval starts at the block's largest Ritz value, which
     must not be a wanted one) */
  if (n < 1 || nev < 1 || nex < 0 || k > n || (nex == 0 && nev < n) || !(tol > 0.0) || kw < 0 || kw > k)
    return info->status = -1;
  cplx* L = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)n);
  cplx* A = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)n);
  cplx* Y = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)k);
  cplx* Q = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)k);
  cplx* F = (cplx*)malloc(sizeof(cplx) * (size_t)n * (size_t)k);
  cplx* v0 = (cplx*)malloc(sizeof(cplx) * (size_t)n);
  double* mu = (double*)malloc(sizeof(double) * (size_t)k);
  double* rho = (double*)malloc(sizeof(double) * (size_t)k);
  double* lam = (double*)malloc(sizeof(double) * (size_t)k);
  int64_t bad = orc_cholesky(n, S, lds, L, n);
  if (bad) {
    info->status = -2;
    info->bad_column = (int32_t)(bad - 1);
    goto done;
  }
  orc_reduce(n, H, ldh, L, n, A, n);
  {
    double lz[3];
    orc_gauss_block(opt->seed, 1u, n, 1, 0, v0, n);
    orc_lanczos(n, A, n, opt->lanczos_steps, v0, lz);
    info->theta_min = lz[0];
    info->b_upper = lz[2];
    orc_gauss_block(opt->seed, 2u, n, 1, 0, v0, n);
    orc_lanczos(n, H, ldh, opt->lanczos_steps, v0, lz);
    info->h_H = fabs(lz[0]) > fabs(lz[1]) ? fabs(lz[0]) : fabs(lz[1]);
  }
  /* start block */
  if (V_warm && kw > 0) orc_lh_times(n, kw, L, n, V_warm, ldv, Y, n);
  if (kw < k) orc_gauss_block(opt->seed, 3u, n, k - kw, kw, &Y[(size_t)kw * n], n);
  orc_householder_qr(n, k, Y, n, Q, n, NULL, 0);
  memcpy(Y, Q, sizeof(cplx) * (size_t)n * (size_t)k);
  double a0, a, b = info->b_upper;
  if (opt->have_bounds && bounds_in) {
    a0 = bounds_in[0];
    a = bounds_in[1];
  } else {
    orc_rayleigh_ritz(n, A, n, Y, n, k, mu);
    a0 = info->theta_min < mu[0] ? info->theta_min : mu[0];
    a = mu[k - 1];
  }
  int64_t c = 0;
  int32_t it = 0;
  double hs = tol * info->h_H;
  info->status = -3;
  for (it = 1; it <= opt->max_iter; it++) {
    int64_t ka = k - c;
    /* the damped interval [a, b] must not be empty: with the block spanning
       the space and an exact Lanczos bound (n at most its steps) b equals a */
    {
      double scale = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
      if (info->h_H > scale) scale = info->h_H;
      if (scale < 1e-300) scale = 1e-300;
      if (b < a + 1e-8 * scale) b = a + 1e-8 * scale;
    }
    orc_filter(n, A, n, &Y[(size_t)c * n], n, ka, opt->degree, a, b, a0);
    info->filter_flops += 8.0 * (double)n * (double)n * (double)ka * (double)opt->degree;
    /* QR of [Y_lock | Y_active] on a copy (the factorization overwrites its
       input); the locked columns stay as they were and the active block
       becomes Q(:, c:k) */
    memcpy(F, Y, sizeof(cplx) * (size_t)n * (size_t)k);
    orc_householder_qr(n, k, F, n, Q, n, NULL, 0);
    memcpy(&Y[(size_t)c * n], &Q[(size_t)c * n], sizeof(cplx) * (size_t)n * (size_t)ka);
    orc_rayleigh_ritz(n, A, n, &Y[(size_t)c * n], n, ka, mu);
    orc_residuals(n, A, n, L, n, &Y[(size_t)c * n], n, ka, mu, rho);
    int64_t nl = 0;
    while (c + nl < nev && nl < ka && rho[nl] <= hs) {
      lam[c + nl] = mu[nl];
      nl++;
    }
    c += nl;
    a = mu[ka - 1];
    if (mu[0] < a0) a0 = mu[0];
    for (int64_t j = 0; j < ka - nl; j++) lam[c + j] = mu[nl + j];
    info->converged = (int32_t)c;
    if (c >= nev) { info->status = 0; break; }
  }
  info->iterations = it > opt->max_iter ? opt->max_iter : it;
  info->a0 = a0;
  info->a = a;
  /* outputs: the converged prefix (all nev on success) */
  {
    int64_t nout = info->status == 0 ? nev : c;
    for (int64_t j = 0; j < nev; j++) evals[j] = j < nout ? lam[j] : NAN;
    if (X) {
      for (int64_t j = 0; j < nev; j++)
        for (int64_t i = 0; i < n; i++) AT(X, ldx, i, j) = Y[(size_t)i + (size_t)j * n];
      orc_backtransform(n, nev, L, n, X, ldx);
      /* generalized residuals relative to h_H */
      double* r2 = (double*)malloc(sizeof(double) * (size_t)nev);
      orc_residuals(n, A, n, L, n, Y, n, nev, lam, r2);
      double mx = 0.0;
      for (int64_t j = 0; j < nout; j++) if (r2[j] / info->h_H > mx) mx = r2[j] / info->h_H;
      info->max_rel_residual = mx;
      free(r2);
    }
    if (Y_state) memcpy(Y_state, Y, sizeof(cplx) * (size_t)n * (size_t)k);
  }
done:
  free(L); free(A); free(Y); free(Q); free(F); free(v0); free(mu); free(rho); free(lam);
  return info->status;
}
