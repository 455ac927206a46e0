/*
 * Memory- and undefined-behaviour check of the CPU oracle: this driver is
 * compiled together with oracle/chfsi_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only) by tests/test_host_cpu.py and
 * runs every path of the oracle's solve on a small problem: a cold solve, a
 * warm solve with the previous vectors and bounds, a solve that stops at the
 * iteration limit, an S that is not positive definite and invalid sizes.
 *
 * The problem is built here with a known spectrum (A = Q diag(lambda) Q^H,
 * Q a product of Householder reflectors, S = L L^H with L unit lower
 * triangular, H = L A L^H), so the run also checks that the cold solve
 * returns the smallest eigenvalues.  Exit status 0 on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double re, im; } cplx;
typedef struct {
  int32_t degree, max_iter, lanczos_steps, have_bounds;
  uint64_t seed;
} orc_opts;
typedef struct {
  int32_t iterations, converged, status, bad_column;
  double b_upper, theta_min, h_H, a0, a, filter_flops, max_rel_residual;
} orc_info;

int32_t orc_solve(int64_t n, const cplx* H, int64_t ldh, const cplx* S, int64_t lds, int64_t nev, int64_t nex,
                  const cplx* V_warm, int64_t ldv, int64_t kw, const double* bounds_in, double tol, const orc_opts* opt,
                  double* evals, cplx* X, int64_t ldx, cplx* Y_state, orc_info* info);
void orc_gauss_block(uint64_t seed, uint32_t stream, int64_t n, int64_t k, int64_t col0, cplx* Y, int64_t ldy);

#define N 40
#define NEV 6
#define NEX 3

static cplx cm(cplx a, cplx b) { cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static cplx cj(cplx a) { cplx r = {a.re, -a.im}; return r; }

/* C = A B^H (n x n, column-major) */
static void mul_bh(const cplx* A, const cplx* B, cplx* C) {
  for (int j = 0; j < N; j++)
    for (int i = 0; i < N; i++) {
      cplx s = {0, 0};
      for (int l = 0; l < N; l++) {
        cplx t = cm(A[i + l * N], cj(B[j + l * N]));
        s.re += t.re;
        s.im += t.im;
      }
      C[i + j * N] = s;
    }
}

static int cmp_d(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return x < y ? -1 : x > y;
}

int main(void) {
  static cplx Q[N * N], T[N * N], A[N * N], L[N * N], S[N * N], H[N * N], G[N * N], X[N * NEV], V[N];
  double lam[N], sorted[N], ev[NEV];
  /* spectrum: a cluster near -1, the rest spread up to 50 */
  for (int i = 0; i < N; i++) lam[i] = i < 4 ? -1.0 + 1e-3 * i : 0.5 + 1.3 * (double)((i * 7) % N);
  /* Q = product of three Householder reflectors I - 2 v v^H / (v^H v) */
  memset(Q, 0, sizeof Q);
  for (int i = 0; i < N; i++) Q[i + i * N].re = 1.0;
  for (int r = 0; r < 3; r++) {
    orc_gauss_block(11, 40u + (uint32_t)r, N, 1, 0, V, N);
    double vv = 0;
    for (int i = 0; i < N; i++) vv += V[i].re * V[i].re + V[i].im * V[i].im;
    for (int j = 0; j < N; j++) {
      cplx d = {0, 0}; /* v^H q_j */
      for (int i = 0; i < N; i++) {
        cplx t = cm(cj(V[i]), Q[i + j * N]);
        d.re += t.re;
        d.im += t.im;
      }
      for (int i = 0; i < N; i++) {
        cplx t = cm(V[i], d);
        Q[i + j * N].re -= 2.0 * t.re / vv;
        Q[i + j * N].im -= 2.0 * t.im / vv;
      }
    }
  }
  for (int j = 0; j < N; j++)
    for (int i = 0; i < N; i++) {
      T[i + j * N].re = Q[i + j * N].re * lam[j];
      T[i + j * N].im = Q[i + j * N].im * lam[j];
    }
  mul_bh(T, Q, A); /* Q diag(lambda) Q^H */
  orc_gauss_block(12, 50u, N, N, 0, L, N);
  for (int j = 0; j < N; j++)
    for (int i = 0; i < N; i++) {
      if (i < j) { L[i + j * N].re = 0; L[i + j * N].im = 0; }
      else if (i == j) { L[i + j * N].re = 1; L[i + j * N].im = 0; }
      else { L[i + j * N].re *= 0.05 / sqrt((double)N); L[i + j * N].im *= 0.05 / sqrt((double)N); }
    }
  mul_bh(L, L, S);
  /* H = L A L^H: T = L A, H = T L^H */
  for (int j = 0; j < N; j++)
    for (int i = 0; i < N; i++) {
      cplx s = {0, 0};
      for (int l = 0; l < N; l++) {
        cplx t = cm(L[i + l * N], A[l + j * N]);
        s.re += t.re;
        s.im += t.im;
      }
      T[i + j * N] = s;
    }
  mul_bh(T, L, H);
  for (int j = 0; j < N; j++) /* exactly Hermitian */
    for (int i = 0; i <= j; i++) {
      cplx h = {(H[i + j * N].re + H[j + i * N].re) / 2, (H[i + j * N].im - H[j + i * N].im) / 2};
      H[i + j * N] = h;
      H[j + i * N] = cj(h);
      cplx s = {(S[i + j * N].re + S[j + i * N].re) / 2, (S[i + j * N].im - S[j + i * N].im) / 2};
      S[i + j * N] = s;
      S[j + i * N] = cj(s);
    }
  memcpy(sorted, lam, sizeof lam);
  qsort(sorted, N, sizeof(double), cmp_d);

  orc_opts o = {8, 1000, 10, 0, 3};
  orc_info info;
  static cplx Ys[N * (NEV + NEX)];
  if (orc_solve(N, H, N, S, N, NEV, NEX, NULL, N, 0, NULL, 1e-10, &o, ev, X, N, Ys, &info) != 0) {
    fprintf(stderr, "cold solve failed: status %d\n", info.status);
    return 1;
  }
  for (int i = 0; i < NEV; i++)
    if (fabs(ev[i] - sorted[i]) > 1e-9 * 50.0) {
      fprintf(stderr, "eigenvalue %d: %.17g against %.17g\n", i, ev[i], sorted[i]);
      return 1;
    }
  /* warm solve from the previous vectors and bounds */
  double bounds[2] = {info.a0, info.a};
  orc_opts ow = o;
  ow.have_bounds = 1;
  static cplx X2[N * NEV];
  double ev2[NEV];
  if (orc_solve(N, H, N, S, N, NEV, NEX, X, N, NEV, bounds, 1e-10, &ow, ev2, X2, N, NULL, &info) != 0) {
    fprintf(stderr, "warm solve failed: status %d\n", info.status);
    return 1;
  }
  /* iteration limit: status -3 with the converged prefix */
  orc_opts o1 = o;
  o1.max_iter = 1;
  int32_t st = orc_solve(N, H, N, S, N, NEV, NEX, NULL, N, 0, NULL, 1e-10, &o1, ev2, X2, N, NULL, &info);
  if (st != -3 && st != 0) {
    fprintf(stderr, "limited solve: status %d\n", st);
    return 1;
  }
  /* S not positive definite */
  memcpy(G, S, sizeof S);
  G[5 + 5 * N].re = -1.0;
  if (orc_solve(N, H, N, G, N, NEV, NEX, NULL, N, 0, NULL, 1e-10, &o, ev2, X2, N, NULL, &info) != -2 ||
      info.bad_column != 5) {
    fprintf(stderr, "not positive definite: status %d column %d\n", info.status, info.bad_column);
    return 1;
  }
  /* invalid sizes */
  if (orc_solve(N, H, N, S, N, NEV, N, NULL, N, 0, NULL, 1e-10, &o, ev2, X2, N, NULL, &info) != -1) {
    fprintf(stderr, "invalid sizes accepted\n");
    return 1;
  }
  printf("oracle sanitizer run ok\n");
  return 0;
}
