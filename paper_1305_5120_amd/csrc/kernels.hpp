// Launchers of the non-GEMM kernels of the ChFSI library.
#pragma once

#include "common.hpp"

namespace chfsi {

// ---- random start vectors: Philox4x32-10 + Box-Muller ---------------------
// Y(i, j) = complex Gaussian number (i + (j + col0) * n) of `stream` under `seed`.
void random_block(uint64_t seed, uint32_t stream, int64_t n, int64_t k, int64_t col0, zc* Y, int64_t ldy, hipStream_t st);
// Raw Philox blocks, for known-answer checks: ctr/key/out are device arrays of
// 4*count, 2*count, 4*count uint32.
void philox_raw(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count, hipStream_t st);

// ---- elementwise / layout --------------------------------------------------
void fill_i32(int* p, int64_t count, int v, hipStream_t st);
void copy2d(const zc* src, int64_t lds, zc* dst, int64_t ldd, int64_t m, int64_t n, hipStream_t st);
// out = a X + b Y (m x n, real a and b)
void lincomb2d(double a, const zc* X, int64_t ldx, double b, const zc* Y, int64_t ldy, zc* out, int64_t ldo, int64_t m,
               int64_t n, hipStream_t st);
// precision conversions of an m x n block (round to nearest / exact widening)
void to_f32(const zc* src, int64_t lds, cc* dst, int64_t ldd, int64_t m, int64_t n, hipStream_t st);
void to_f64(const cc* src, int64_t lds, zc* dst, int64_t ldd, int64_t m, int64_t n, hipStream_t st);
// The filter on the Ritz residual (m x n blocks, mu device FP64): per
// column j, s_j = the power of two at or above max |AY0 - Y0 mu| (1 for a
// zero column) into scale[j], R = (FP32) ((AY0 - Y0 diag(mu)) / s_j) and
// D1 = (FP32) (alpha0 (AY0 - Y0 diag(mu)) / s_j); then
// F = Y0 diag(t) + D diag(scale) (t, scale device FP64, n entries)
void ritz_forcing(const zc* Y0, int64_t ldy, const zc* AY0, int64_t lday, const double* mu, double alpha0, cc* R,
                  int64_t ldr, cc* D1, int64_t ldd, double* scale, int64_t m, int64_t n, hipStream_t st);
void ritz_combine(const zc* Y0, int64_t ldy, const double* t, const double* scale, const cc* D, int64_t ldd, zc* F,
                  int64_t ldf, int64_t m, int64_t n, hipStream_t st);
void set_identity(zc* Y, int64_t ldy, int64_t m, int64_t n, hipStream_t st);
void zero_strict_upper(zc* A, int64_t lda, int64_t n, hipStream_t st);
// A <- the Hermitian matrix whose lower triangle A holds (upper triangle
// overwritten by the conjugate transpose, diagonal made real)
void hermitian_from_lower(zc* A, int64_t lda, int64_t n, hipStream_t st);
// R(:, j) = W(:, j) - mu[j] Y(:, j)
void residual_block(const zc* W, int64_t ldw, const zc* Y, int64_t ldy, const double* mu, zc* R, int64_t ldr, int64_t n,
                    int64_t k, hipStream_t st);
// out[j] = ||R(:, j)||_2
void column_norms(const zc* R, int64_t ldr, int64_t n, int64_t k, double* out, hipStream_t st);
// out[0] = max_j |L(j,j)| / min_j |L(j,j)| (+inf for a zero or non-finite
// diagonal entry): a lower bound on the condition number of triangular L
void diag_ratio(const zc* L, int64_t ld, int64_t k, double* out, hipStream_t st);
// flag[0] = 1 if any entry of the n x k block is not finite (else untouched)

// ---- Cholesky --------------------------------------------------------------
// Factor the nb x nb diagonal block W(j0:j0+nb, j0:j0+nb) (lower triangle
// read) into L's block and its inverse into Linv's block.  On a pivot that
// is not positive, info[0] receives min(info[0], j0 + column + 1) (info is
// initialised to a huge value by the caller).
void chol_diag(const zc* W, int64_t ldw, zc* L, int64_t ldl, zc* Linv, int64_t ldi, int64_t j0, int64_t nb, int* info,
               hipStream_t st);
constexpr int CHOL_NB = 64;
// Outer block of the two-level blocked Cholesky (columns; a multiple of CHOL_NB).
constexpr int CHOL_NB_OUTER = 256;

// ---- Householder QR --------------------------------------------------------
constexpr int HH_NB = 32;
struct HHPanel {
  zc* F; int64_t ldf; int64_t n;  // matrix being factored (n rows)
  int64_t j0, j1;                 // panel columns [j0, j1)
  int nblk;                       // workgroups (row blocks)
  int64_t rows_per_blk;           // multiple of 256
  zc* part;                       // 2 x nblk x HH_NB partial sums
  zc* top;                        // 2 x HH_NB top rows
  zc* tau;                        // k reflector scalars
};
void hh_panel_setup(HHPanel& p);
void hh_first_partials(const HHPanel& p, hipStream_t st);
void hh_column(const HHPanel& p, int64_t j, hipStream_t st);
// Vp(0:n-j0, 0:nb): explicit unit lower-trapezoidal V of the panel
void hh_extract_v(const zc* F, int64_t ldf, int64_t n, int64_t j0, int64_t j1, zc* Vp, int64_t ldv, hipStream_t st);
// T (nb x nb, ld nb) of H_j0 ... H_{j1-1} = I - V T V^H from the Gram V^H V
void hh_build_t(const zc* gram, const zc* tau, int64_t cnt, zc* T, hipStream_t st);

// ---- Jacobi eigensolver for Hermitian k x k --------------------------------
constexpr int JACOBI_LDS_MAX = 96;
// Single-workgroup solver (k <= JACOBI_LDS_MAX): w ascending, Z (ld ldz).
// tau: couplings |G(p,q)| <= tau count as converged (0: working accuracy)
void jacobi_small(const zc* G, int64_t ldg, int64_t k, double* w, zc* Z, int64_t ldz, zc* Ztmp, int* sweeps_out,
                  hipStream_t st, double tau = 0.0);
// Multi-launch pieces for larger k.
void jacobi_init(const zc* G, int64_t ldg, int64_t k, zc* G0, zc* Z0, hipStream_t st);
// out[0] = sum |G_ij|^2 off the diagonal, out[1] = sum over all (two-stage)
void jacobi_norms(const zc* G, int64_t k, double* part, double* out, hipStream_t st);
void jacobi_sort(const zc* G, const zc* Z, int64_t k, double* w, int* rank, zc* Zout, int64_t ldz, hipStream_t st);
// Sparse sweeps: count / list the pairs with |G(i,j)|^2 > max(thr_factor *
// fro2, tau^2) (i > j, per column j) and, when ratio > 0, |G(i,j)| > ratio *
// |G(i,i) - G(j,j)|; then apply one round of disjoint pairs in place.
void jacobi_count(const zc* G, int64_t k, const double* fro2, double thr_factor, double tau, double ratio, int* counts,
                  hipStream_t st);
void jacobi_list(const zc* G, int64_t k, const double* fro2, double thr_factor, double tau, double ratio,
                 const int* offsets, int* pairs, hipStream_t st);
// pairs: 2 np ints (p < q); pairof: k ints, the pair index of each row or -1
void jacobi_sparse_round(zc* G, zc* Z, int64_t k, const int* pairs, int np, const int* pairof, void* prm_scratch,
                         const double* fro2, double tau, int* rotated, hipStream_t st);
size_t jacobi_rot_bytes();
// One round of the block-ordered Jacobi sweep on G (k x k, ld k, Hermitian,
// in place) with its rotations accumulated into Z (k x k, ld k, in place);
// V: block_jacobi_v_bytes(k) of device scratch; rounds 0 .. block_jacobi_rounds(k) - 1
// make a sweep; *rotated set when a rotation was applied.
size_t block_jacobi_v_bytes(int64_t k);
int64_t block_jacobi_rounds(int64_t k);
void block_jacobi_round(zc* G, zc* Z, int64_t k, int64_t round, const double* fro2, double tau, zc* V, int* rotated,
                        hipStream_t st);

// ---- Eigenvector refinement for nearly diagonal Hermitian k x k -------------
// One step's coefficients E (k x k) from S = X^H G X and P = X^H X, both
// read as their Hermitian parts (P null: X = I, then also Xout = I + E);
// lam = Rayleigh quotients; *corr (zero at launch) = max off-diagonal |E| as
// double bits; *corr_next (nullable) is zeroed for the next step.
void refine_coeffs(const zc* S, const zc* P, int64_t k, double tau, zc* E, zc* Xout, double* lam,
                   unsigned long long* corr, unsigned long long* corr_next, hipStream_t st);
// w ascending = lam sorted; Zout (ld ldz) = Z's columns in that order
void sort_by_values(const double* lam, const zc* Z, int64_t k, double* w, int* rank, zc* Zout, int64_t ldz,
                    hipStream_t st);

// ---- Lanczos pieces ---------------------------------------------------------
// y = A x (A n x n, lda); part: work of JMV_SPLITS * n
void zgemv(const zc* A, int64_t lda, int64_t n, const zc* x, zc* y, zc* part, hipStream_t st);
// out[p] = V(:, p)^H w for p < cnt
void multi_dot(const zc* V, int64_t ldv, int64_t n, int64_t cnt, const zc* w, zc* out, hipStream_t st);
// w -= V(:, 0:cnt) h
void sub_combination(const zc* V, int64_t ldv, int64_t n, int64_t cnt, const zc* h, zc* w, hipStream_t st);
// w -= alpha[j] v_j + beta[j] v_{j-1}; alpha[j] = Re(h[0]) read from device
void lanczos_three_term(zc* w, const zc* V, int64_t ldv, int64_t n, int64_t j, double* alpha, const double* beta,
                        const zc* h, hipStream_t st);
// beta_out = ||w||, v = w / beta (0 if beta == 0)
void normalize(const zc* w, int64_t n, zc* v, double* beta_out, hipStream_t st);

}  // namespace chfsi
