// Non-GEMM kernels of the ChFSI library (gfx950): start vectors, Cholesky
// diagonal blocks, Householder column steps, the Jacobi eigensolver of the
// Rayleigh-Ritz step, residual norms and the Lanczos pieces.  All of these are
// latency- or bandwidth-bound; the dense products live in zgemm.hip.
#include "kernels.hpp"

#include <mutex>

namespace chfsi {

namespace {

constexpr int NT = 256;

inline dim3 grid1(int64_t total, int nt = NT) { return dim3((unsigned)std::max<int64_t>(1, cdiv(total, nt))); }

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC 2011) and Box-Muller Gaussians
// --------------------------------------------------------------------------
__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; r++) {
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t y0 = hi1 ^ c[1] ^ k0, y2 = hi0 ^ c[3] ^ k1;
    c[0] = y0; c[1] = lo1; c[2] = y2; c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__global__ void k_philox_raw(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  uint32_t c[4] = {ctr[4 * e], ctr[4 * e + 1], ctr[4 * e + 2], ctr[4 * e + 3]};
  philox10(c, key[2 * e], key[2 * e + 1]);
  for (int i = 0; i < 4; i++) out[4 * e + i] = c[i];
}

__global__ void k_random_block(uint64_t seed, uint32_t stream, int64_t n, int64_t k, int64_t col0, zc* Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int64_t i = e % n, j = e / n;
  const uint64_t idx = (uint64_t)i + (uint64_t)(j + col0) * (uint64_t)n;
  uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), stream, 0u};
  philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t q1 = (((uint64_t)c[0] << 32) | c[1]) >> 11;
  const uint64_t q2 = (((uint64_t)c[2] << 32) | c[3]) >> 11;
  const double u1 = ((double)q1 + 0.5) * 0x1p-53;
  const double u2 = ((double)q2 + 0.5) * 0x1p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double t = 6.283185307179586476925286766559 * u2;
  Y[i + j * ldy] = zmk(r * cos(t), r * sin(t));
}

// --------------------------------------------------------------------------
// elementwise
// --------------------------------------------------------------------------
__global__ void k_fill_i32(int* p, int64_t count, int v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = v;
}

__global__ void k_copy2d(const zc* src, int64_t lds, zc* dst, int64_t ldd, int64_t m, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  const int64_t i = e % m, j = e / m;
  dst[i + j * ldd] = src[i + j * lds];
}

// out = a X + b Y (real a, b; m x n blocks)
__global__ void k_lincomb2d(double a, const zc* X, int64_t ldx, double b, const zc* Y, int64_t ldy, zc* out,
                            int64_t ldo, int64_t m, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  const int64_t i = e % m, j = e / m;
  const zc x = X[i + j * ldx], y = Y[i + j * ldy];
  out[i + j * ldo] = zmk(fma(a, x.x, b * y.x), fma(a, x.y, b * y.y));
}

__global__ void k_z2c(const zc* src, int64_t lds, cc* dst, int64_t ldd, int64_t m, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  const int64_t i = e % m, j = e / m;
  const zc v = src[i + j * lds];
  dst[i + j * ldd] = make_float2((float)v.x, (float)v.y);
}

__global__ void k_c2z(const cc* src, int64_t lds, zc* dst, int64_t ldd, int64_t m, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  const int64_t i = e % m, j = e / m;
  const cc v = src[i + j * lds];
  dst[i + j * ldd] = make_double2((double)v.x, (double)v.y);
}

// The filter on the Ritz residual: with Y_0 Ritz vectors (values mu), the
// residual R = A Y_0 - Y_0 diag(mu) of column j (one workgroup) formed in
// FP64, scaled by the power of two s_j at or above its largest entry (1 for
// a zero column; the scaling is exact) and rounded to FP32, with the residual
// part's first iterate D_1 = alpha0 R / s_j (the first degree step of eq. (2)
// applied to Y_0); scale[j] = s_j.
__global__ void __launch_bounds__(256) k_ritz_forcing(const zc* Y0, int64_t ldy, const zc* AY0, int64_t lday,
                                                      const double* mu, double alpha0, cc* R, int64_t ldr, cc* D1,
                                                      int64_t ldd, double* scale, int64_t m) {
  __shared__ double red[4];
  const int64_t j = blockIdx.x;
  const zc* y = Y0 + j * ldy;
  const zc* w = AY0 + j * lday;
  const double mj = mu[j];
  double mx = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const zc yv = y[i], wv = w[i];
    mx = fmax(mx, fmax(fabs(fma(-mj, yv.x, wv.x)), fabs(fma(-mj, yv.y, wv.y))));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  int ex = 0;
  (void)frexp(mx, &ex);
  const double sc = mx > 0.0 ? ldexp(1.0, ex) : 1.0;
  const double inv = 1.0 / sc;
  if (threadIdx.x == 0) scale[j] = sc;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const zc yv = y[i], wv = w[i];
    const double rx = fma(-mj, yv.x, wv.x) * inv, ry = fma(-mj, yv.y, wv.y) * inv;
    R[i + j * ldr] = make_float2((float)rx, (float)ry);
    D1[i + j * ldd] = make_float2((float)(alpha0 * rx), (float)(alpha0 * ry));
  }
}

// The filtered block from its two parts: F = Y_0 diag(t) + D diag(scale)
// (D widened).
__global__ void k_ritz_combine(const zc* Y0, int64_t ldy, const double* t, const double* scale, const cc* D,
                               int64_t ldd, zc* F, int64_t ldf, int64_t m, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  const int64_t i = e % m, j = e / m;
  const zc y = Y0[i + j * ldy];
  const cc d = D[i + j * ldd];
  const double tj = t[j], sj = scale[j];
  F[i + j * ldf] = zmk(fma(tj, y.x, sj * (double)d.x), fma(tj, y.y, sj * (double)d.y));
}

__global__ void k_set_identity(zc* Y, int64_t ldy, int64_t m, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * n) return;
  const int64_t i = e % m, j = e / m;
  Y[i + j * ldy] = zmk(i == j ? 1.0 : 0.0, 0.0);
}

__global__ void k_zero_strict_upper(zc* A, int64_t lda, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int64_t i = e % n, j = e / n;
  if (i < j) A[i + j * lda] = zmk(0.0, 0.0);
}

__global__ void k_hermitian_from_lower(zc* A, int64_t lda, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int64_t i = e % n, j = e / n;
  if (i < j) return;
  if (i == j) A[i + i * lda].y = 0.0;
  else A[j + i * lda] = zconj(A[i + j * lda]);
}

__global__ void k_residual(const zc* W, int64_t ldw, const zc* Y, int64_t ldy, const double* mu, zc* R, int64_t ldr, int64_t n,
                           int64_t k) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * k) return;
  const int64_t i = e % n, j = e / n;
  R[i + j * ldr] = zsub(W[i + j * ldw], zscale(mu[j], Y[i + j * ldy]));
}

__global__ void k_column_norms(const zc* R, int64_t ldr, int64_t n, double* out) {
  __shared__ double red[16];
  const int64_t j = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += zabs2(R[i + j * ldr]);
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[j] = sqrt(s);
}

// Ratio of the largest to the smallest diagonal entry of a triangular factor
// (real, positive diagonal): a lower bound on its condition number.  One
// workgroup; +inf when a diagonal entry is zero or not finite.
__global__ void __launch_bounds__(256) k_diag_ratio(const zc* L, int64_t ld, int64_t k, double* out) {
  __shared__ double smax[256], smin[256];
  double mx = 0.0, mn = INFINITY;
  bool bad = false;
  for (int64_t j = threadIdx.x; j < k; j += blockDim.x) {
    const double d = fabs(L[j + j * ld].x);
    if (!(d > 0.0) || !isfinite(d)) bad = true;
    mx = fmax(mx, d);
    mn = fmin(mn, d);
  }
  smax[threadIdx.x] = bad ? INFINITY : mx;
  smin[threadIdx.x] = mn;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = isfinite(smax[0]) && smin[0] > 0.0 ? smax[0] / smin[0] : INFINITY;
}

// --------------------------------------------------------------------------
// Cholesky diagonal block (nb <= 64) and the inverse of its factor, one
// workgroup, the block in LDS (rows beyond nb padded with the identity).
//
// Factorization, right-looking in panels of CPW columns: wave 0 factors the
// panel (lane r holds row r of it in registers; the pivot and the panel
// entries a column update needs come from other lanes by readlane, the
// pivot's inverse square root from the hardware estimate and two Newton
// steps), then all waves apply the rank-CPW update to the trailing lower
// triangle.  The sequential chain per pivot is a few register operations,
// not a workgroup barrier.
//
// Inverse X = L^{-1} by recursive doubling: with X's diagonal blocks of size
// s known, each pair of them gives the block below as -C^{-1} (B A^{-1}) for
// L = [A 0; B C]; six levels s = 1, 2, ..., 32, each two small products
// computed by all threads.  The sums run over whole blocks (the strictly
// upper parts of A^{-1} and C^{-1} are zero), so every loop has a fixed trip
// count and unrolls: 16 waves, four per SIMD, keep the LDS loads in flight.
// --------------------------------------------------------------------------
constexpr int CNB = CHOL_NB;
constexpr int CLD = CNB + 1;  // LDS row stride (complex); keeps 16-lane groups on distinct banks
constexpr int CPW = 8;        // panel width
constexpr int CNT = 1024;     // threads of the diagonal-block kernel
constexpr int CWV = CNT / 64; // its waves

__device__ __forceinline__ double lane_read(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// One doubling level of the inverse (block size SZ): for each of the
// CNB / (2 SZ) pairs at origin o, X(o+SZ.., o..) = -C^{-1} (B A^{-1}) with
// B = L(o+SZ.., o..), A^{-1} = X(o.., o..), C^{-1} = X(o+SZ.., o+SZ..).
template <int SZ>
__device__ __forceinline__ void chol_inv_level(const zc* S, zc* X, zc* T, int tid) {
  constexpr int PER = SZ * SZ, TOTAL = (CNB / (2 * SZ)) * PER;
  for (int e = tid; e < TOTAL; e += CNT) {
    const int pair = e / PER, rem = e % PER, i = rem / SZ, j = rem % SZ, o = 2 * SZ * pair;
    const zc* brow = S + (o + SZ + i) * CLD + o;
    const zc* acol = X + o * CLD + o + j;
    zc acc = zmk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < SZ; k++) {
      const zc bv = brow[k], av = acol[k * CLD];
      acc = zmk(fma(bv.x, av.x, fma(-bv.y, av.y, acc.x)), fma(bv.x, av.y, fma(bv.y, av.x, acc.y)));
    }
    T[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < TOTAL; e += CNT) {
    const int pair = e / PER, rem = e % PER, i = rem / SZ, j = rem % SZ, o = 2 * SZ * pair;
    const zc* crow = X + (o + SZ + i) * CLD + o + SZ;
    const zc* tcol = T + pair * PER + j;
    zc acc = zmk(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < SZ; k++) {
      const zc cv = crow[k], tv = tcol[k * SZ];
      acc = zmk(fma(cv.x, tv.x, fma(-cv.y, tv.y, acc.x)), fma(cv.x, tv.y, fma(cv.y, tv.x, acc.y)));
    }
    X[(o + SZ + i) * CLD + o + j] = zmk(-acc.x, -acc.y);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(CNT) k_chol_diag(const zc* W, int64_t ldw, zc* L, int64_t ldl, zc* Linv, int64_t ldi,
                                                    int64_t j0, int nb, int* info) {
  static_assert(CNB == 64 && CNB % CPW == 0 && CNB % CWV == 0, "64 x 64 blocks, whole panels");
  constexpr int CPT = CNB / CWV;  // columns per thread in the element-wise loops
  extern __shared__ zc smem[];
  zc* S = smem;                // S[r * CLD + c]: the matrix, then L (lower triangle)
  zc* X = smem + CNB * CLD;    // X[r * CLD + c]: L^{-1} (lower triangle, zero above)
  zc* T = X + CNB * CLD;       // scratch of the inverse: up to CNB * CNB / 4 entries
  __shared__ int failed;
  const int tid = threadIdx.x;
  const int r = tid & 63;
  const int q = __builtin_amdgcn_readfirstlane(tid >> 6);
#pragma unroll
  for (int t = 0; t < CPT; t++) {
    const int c = q + CWV * t;
    zc v = zmk(r == c ? 1.0 : 0.0, 0.0);
    if (r < nb && c < nb) v = r >= c ? W[(j0 + r) + (j0 + c) * ldw] : zmk(0.0, 0.0);
    S[r * CLD + c] = v;
    X[r * CLD + c] = zmk(0.0, 0.0);
  }
  if (tid == 0) failed = -1;
  __syncthreads();

  for (int jb = 0; jb < CNB; jb += CPW) {
    if (q == 0) {
      zc p[CPW];
#pragma unroll
      for (int i = 0; i < CPW; i++) p[i] = S[r * CLD + jb + i];
      // Branch-free pivot steps (selects, no divergent blocks on the chain
      // of 64 dependent pivots); after a non-positive pivot the panel goes
      // on with a unit stand-in and the failure is reported instead.
      int fail = -1;    // first column of the panel without a positive pivot (uniform)
      double xd = 0.0;  // lane r in the panel: 1 / l(r, r)
#pragma unroll
      for (int i = 0; i < CPW; i++) {
        const int j = jb + i;
        const double d0 = lane_read(p[i].x, j);
        const bool good = d0 > 0.0;
        fail = (fail < 0 && !good) ? j : fail;
        const double d = good ? d0 : 1.0;
        double y = __builtin_amdgcn_rsq(d);
        y = y * fma(-0.5 * d * y, y, 1.5);
        y = y * fma(-0.5 * d * y, y, 1.5);
        // rows below the pivot scale by 1 / l(j, j), the pivot row becomes
        // l(j, j) = d y, rows above zero
        const double f = r > j ? y : 0.0;
        const double dg = r == j ? d * y : 0.0;
        p[i] = zmk(fma(f, p[i].x, dg), f * p[i].y);
        xd = r == j ? y : xd;
#pragma unroll
        for (int ii = i + 1; ii < CPW; ii++) {
          // p[ii] -= p[i] conj(l(jb + ii, j))
          const double lx = lane_read(p[i].x, jb + ii), ly = lane_read(p[i].y, jb + ii);
          p[ii] = zmk(fma(-p[i].x, lx, fma(-p[i].y, ly, p[ii].x)), fma(-p[i].y, lx, fma(p[i].x, ly, p[ii].y)));
        }
      }
      if (fail >= 0 && r == 0) failed = fail;
      if (r >= jb && r < jb + CPW) X[r * CLD + r] = zmk(xd, 0.0);  // X's diagonal: 1 / l(r, r)
#pragma unroll
      for (int i = 0; i < CPW; i++) S[r * CLD + jb + i] = p[i];
    }
    __syncthreads();
    if (failed >= 0) break;
    // trailing update: columns c >= jb + CPW, rows r >= c
    if (q + CWV * (CPT - 1) >= jb + CPW) {  // this wave owns a trailing column (uniform)
      zc lr[CPW];
#pragma unroll
      for (int i = 0; i < CPW; i++) lr[i] = S[r * CLD + jb + i];
#pragma unroll
      for (int t = 0; t < CPT; t++) {
        const int c = q + CWV * t;
        if (c >= jb + CPW) {  // uniform over the wave
          zc acc = S[r * CLD + c];
#pragma unroll
          for (int i = 0; i < CPW; i++) {
            const zc lc = S[c * CLD + jb + i];
            acc = zmk(fma(-lr[i].x, lc.x, fma(-lr[i].y, lc.y, acc.x)), fma(-lr[i].y, lc.x, fma(lr[i].x, lc.y, acc.y)));
          }
          if (r >= c) S[r * CLD + c] = acc;
        }
      }
    }
    __syncthreads();
  }
  if (failed >= 0) {
    if (tid == 0) atomicMin(info, (int)(j0 + failed + 1));
    return;
  }
  // L out (the matrix is final)
#pragma unroll
  for (int t = 0; t < CPT; t++) {
    const int c = q + CWV * t;
    if (r < nb && c < nb) L[(j0 + r) + (j0 + c) * ldl] = r >= c ? S[r * CLD + c] : zmk(0.0, 0.0);
  }
  chol_inv_level<1>(S, X, T, tid);
  chol_inv_level<2>(S, X, T, tid);
  chol_inv_level<4>(S, X, T, tid);
  chol_inv_level<8>(S, X, T, tid);
  chol_inv_level<16>(S, X, T, tid);
  chol_inv_level<32>(S, X, T, tid);
#pragma unroll
  for (int t = 0; t < CPT; t++) {
    const int c = q + CWV * t;
    if (r < nb && c < nb) Linv[(j0 + r) + (j0 + c) * ldi] = r >= c ? X[r * CLD + c] : zmk(0.0, 0.0);
  }
}

// --------------------------------------------------------------------------
// Householder panel.  Reflector j: H = I - tau v v^H with v(j) = 1 and
// H^H x = beta e_j, beta real with the sign opposite to Re x(j).  Each
// workgroup owns a fixed block of rows; a launch applies reflector j to the
// panel and, from the updated rows, forms the partial inner products that
// the next column's reflector needs: one launch per column.
//   partial sums  s[c] = sum_{i > j} conj(F(i, j)) F(i, c),  c in [j, j1)
//   top row       F(j, c)
// --------------------------------------------------------------------------
constexpr int HNB = HH_NB;

// Block-reduce acc[0..HNB) (only entries [c0, cnt) meaningful) into dst.
__device__ inline void reduce_partials(zc (&acc)[HNB], int c0, int cnt, zc* dst, double* red /* 4*HNB*2 */) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < HNB; c++) {
    if (c >= c0 && c < cnt) {
      const double re = wave_sum(acc[c].x), im = wave_sum(acc[c].y);
      if (lane == 0) {
        red[(w * HNB + c) * 2] = re;
        red[(w * HNB + c) * 2 + 1] = im;
      }
    }
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < HNB) {
    zc s = zmk(0.0, 0.0);
    if (c >= c0 && c < cnt)
      for (int q = 0; q < (int)(blockDim.x >> 6); q++) s = zadd(s, zmk(red[(q * HNB + c) * 2], red[(q * HNB + c) * 2 + 1]));
    dst[c] = s;
  }
}

__global__ void __launch_bounds__(256) k_hh_first(HHPanel p) {
  __shared__ double red[4 * HNB * 2];
  const int64_t j = p.j0;
  const int cnt = (int)(p.j1 - p.j0);
  const int64_t rbeg = p.j0 + (int64_t)blockIdx.x * p.rows_per_blk;
  const int64_t rend = min(p.n, rbeg + p.rows_per_blk);
  zc acc[HNB];
#pragma unroll
  for (int c = 0; c < HNB; c++) acc[c] = zmk(0.0, 0.0);
  for (int64_t i = rbeg + threadIdx.x; i < rend; i += blockDim.x) {
    const zc* row = p.F + i;
    if (i == j) {
#pragma unroll
      for (int c = 0; c < HNB; c++)
        if (c < cnt) p.top[c] = row[(p.j0 + c) * p.ldf];
    } else if (i > j) {
      const zc x = row[j * p.ldf];
#pragma unroll
      for (int c = 0; c < HNB; c++)
        if (c < cnt) acc[c] = zadd(acc[c], zcmul(x, row[(p.j0 + c) * p.ldf]));
    }
  }
  reduce_partials(acc, 0, cnt, p.part + (int64_t)blockIdx.x * HNB, red);
}

__global__ void __launch_bounds__(256) k_hh_column(HHPanel p, int64_t j) {
  __shared__ double red[4 * HNB * 2];
  __shared__ zc s_tot[HNB], f[HNB];
  __shared__ double sh_beta;
  __shared__ zc sh_scal;
  __shared__ int sh_identity;
  const int cnt = (int)(p.j1 - p.j0);
  const int jl = (int)(j - p.j0);
  const int cur = jl & 1, nxt = cur ^ 1;
  const zc* part_cur = p.part + (int64_t)cur * p.nblk * HNB;
  zc* part_nxt = p.part + (int64_t)nxt * p.nblk * HNB;
  const zc* top_cur = p.top + cur * HNB;
  zc* top_nxt = p.top + nxt * HNB;
  const int tid = threadIdx.x;
  if (tid >= jl && tid < cnt) {
    zc s = zmk(0.0, 0.0);
    for (int b = 0; b < p.nblk; b++) s = zadd(s, part_cur[(int64_t)b * HNB + tid]);
    s_tot[tid] = s;
  }
  __syncthreads();
  if (tid == 0) {
    const zc alpha = top_cur[jl];
    const double xnorm2 = s_tot[jl].x;
    if (xnorm2 == 0.0 && alpha.y == 0.0) {
      sh_identity = 1;
      sh_beta = alpha.x;
      sh_scal = zmk(0.0, 0.0);
      if (blockIdx.x == 0) p.tau[j] = zmk(0.0, 0.0);
      for (int c = jl + 1; c < cnt; c++) f[c] = zmk(0.0, 0.0);
    } else {
      sh_identity = 0;
      const double nrm = sqrt(zabs2(alpha) + xnorm2);
      const double beta = alpha.x >= 0.0 ? -nrm : nrm;
      const zc tau = zmk((beta - alpha.x) / beta, -alpha.y / beta);
      const zc den = zmk(alpha.x - beta, alpha.y);
      const double dd = zabs2(den);
      const zc scal = zmk(den.x / dd, -den.y / dd);  // 1 / (alpha - beta)
      sh_beta = beta;
      sh_scal = scal;
      if (blockIdx.x == 0) p.tau[j] = tau;
      for (int c = jl + 1; c < cnt; c++) {
        // v^H y_c = y_jc + conj(scal) s[c]
        const zc w = zadd(top_cur[c], zcmul(scal, s_tot[c]));
        f[c] = zcmul(tau, w);  // conj(tau) w
      }
    }
  }
  __syncthreads();
  const bool ident = sh_identity != 0;
  const double beta = sh_beta;
  const zc scal = sh_scal;
  const int64_t rbeg = p.j0 + (int64_t)blockIdx.x * p.rows_per_blk;
  const int64_t rend = min(p.n, rbeg + p.rows_per_blk);
  zc acc[HNB];
#pragma unroll
  for (int c = 0; c < HNB; c++) acc[c] = zmk(0.0, 0.0);
  for (int64_t i = rbeg + tid; i < rend; i += blockDim.x) {
    if (i < j) continue;
    zc* row = p.F + i;
    zc vals[HNB];
#pragma unroll
    for (int c = 0; c < HNB; c++)
      if (c >= jl && c < cnt) vals[c] = row[(p.j0 + c) * p.ldf];
    // (register arrays are only indexed with unrolled constants)
    if (!ident) {
      zc xj = zmk(0.0, 0.0);
#pragma unroll
      for (int c = 0; c < HNB; c++)
        if (c == jl) xj = vals[c];
      const zc v = (i == j) ? zmk(1.0, 0.0) : zmul(xj, scal);
      const zc vj = (i == j) ? zmk(beta, 0.0) : v;
#pragma unroll
      for (int c = 0; c < HNB; c++) {
        if (c == jl) vals[c] = vj;
        else if (c > jl && c < cnt) vals[c] = zsub(vals[c], zmul(v, f[c]));
      }
#pragma unroll
      for (int c = 0; c < HNB; c++)
        if (c >= jl && c < cnt) row[(p.j0 + c) * p.ldf] = vals[c];
    }
    if (jl + 1 < cnt) {
      if (i == j + 1) {
#pragma unroll
        for (int c = 0; c < HNB; c++)
          if (c > jl && c < cnt) top_nxt[c] = vals[c];
      } else if (i > j + 1) {
        zc x = zmk(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < HNB; c++)
          if (c == jl + 1) x = vals[c];
#pragma unroll
        for (int c = 0; c < HNB; c++)
          if (c > jl && c < cnt) acc[c] = zadd(acc[c], zcmul(x, vals[c]));
      }
    }
  }
  if (jl + 1 < cnt) reduce_partials(acc, jl + 1, cnt, part_nxt + (int64_t)blockIdx.x * HNB, red);
}

__global__ void k_hh_extract_v(const zc* F, int64_t ldf, int64_t n, int64_t j0, int64_t j1, zc* Vp, int64_t ldv) {
  const int64_t cnt = j1 - j0, rows = n - j0;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cnt) return;
  const int64_t r = e % rows, c = e / rows;
  const int64_t i = j0 + r, col = j0 + c;
  zc v;
  if (i == col) v = zmk(1.0, 0.0);
  else if (i < col) v = zmk(0.0, 0.0);
  else v = F[i + col * ldf];
  Vp[r + c * ldv] = v;
}

__global__ void k_hh_build_t(const zc* gram, const zc* tau, int64_t cnt, zc* T) {
  // gram: cnt x cnt (ld cnt) = V^H V;  T: HNB x HNB column-major (ld HNB), upper
  __shared__ zc Ts[HNB][HNB + 1];
  const int r = threadIdx.x;
  for (int e = r; e < HNB * HNB; e += blockDim.x) Ts[e % HNB][e / HNB] = zmk(0.0, 0.0);
  __syncthreads();
  for (int i = 0; i < (int)cnt; i++) {
    const zc ti = tau[i];
    zc val = zmk(0.0, 0.0);
    if (r < i) {
      zc s = zmk(0.0, 0.0);
      for (int q = r; q < i; q++) s = zadd(s, zmul(Ts[r][q], gram[q + (int64_t)i * cnt]));
      val = zmul(zmk(-ti.x, -ti.y), s);
    }
    __syncthreads();
    if (r < i) Ts[r][i] = val;
    if (r == i) Ts[i][i] = ti;
    __syncthreads();
  }
  for (int e = r; e < HNB * HNB; e += blockDim.x) T[e] = Ts[e % HNB][e / HNB];
}

// --------------------------------------------------------------------------
// Jacobi eigensolver (Hermitian).  Parallel (round-robin) ordering: in each
// round the index pairs are disjoint, so all rotations of a round apply at
// once, G <- J^H G J, Z <- Z J.  Rotation of pair (p, q), p < q, with
// g = G(p, q) = |g| u: real symmetric Jacobi on [[G_pp, |g|], [|g|, G_qq]],
// t = sign(tau)/(|tau| + sqrt(1 + tau^2)), tau = (G_qq - G_pp)/(2|g|),
// c = 1/sqrt(1 + t^2), s = t c, and J = [[u c, u s], [-s, c]] on columns p, q.
// A rotation is skipped when |g|^2 <= 1e-36 ||G||_F^2.
// --------------------------------------------------------------------------
struct Rot {
  double c, s, ur, ui, tg;  // tg = t |g|
  int active;
};

__device__ inline void round_pair(int64_t K2, int64_t round, int64_t t, int64_t& p, int64_t& q) {
  const int64_t a = t, b = K2 - 1 - t;
  auto player = [&](int64_t pos) -> int64_t { return pos == 0 ? 0 : ((pos - 1 + round) % (K2 - 1)) + 1; };
  const int64_t x = player(a), y = player(b);
  p = x < y ? x : y;
  q = x < y ? y : x;
}

__device__ inline Rot make_rot(zc gpp, zc gqq, zc gpq, double skip2) {
  Rot R;
  R.c = 1.0; R.s = 0.0; R.ur = 1.0; R.ui = 0.0; R.tg = 0.0; R.active = 0;
  const double ag2 = zabs2(gpq);
  if (ag2 <= skip2 || ag2 == 0.0) return R;
  const double ag = sqrt(ag2);
  const double tau = (gqq.x - gpp.x) / (2.0 * ag);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  R.c = 1.0 / sqrt(1.0 + t * t);
  R.s = t * R.c;
  R.ur = gpq.x / ag;
  R.ui = gpq.y / ag;
  R.tg = t * ag;
  R.active = 1;
  return R;
}

// 2x2 block update  B <- Jr^H B Js  where J = [[u c, u s], [-s, c]]
__device__ inline void rot_block(const Rot& r, const Rot& s, zc& b00, zc& b01, zc& b10, zc& b11) {
  const zc us = zmk(s.ur, s.ui), ur = zmk(r.ur, r.ui);
  const zc s00 = zscale(s.c, us), s01 = zscale(s.s, us);
  const double s10 = -s.s, s11 = s.c;
  // B Js
  const zc c00 = zadd(zmul(b00, s00), zscale(s10, b01));
  const zc c01 = zadd(zmul(b00, s01), zscale(s11, b01));
  const zc c10 = zadd(zmul(b10, s00), zscale(s10, b11));
  const zc c11 = zadd(zmul(b10, s01), zscale(s11, b11));
  const zc r00 = zscale(r.c, ur), r01 = zscale(r.s, ur);
  const double r10 = -r.s, r11 = r.c;
  // Jr^H (B Js): row0 = conj(r00) row0 + r10 row1 ; row1 = conj(r01) row0 + r11 row1
  b00 = zadd(zcmul(r00, c00), zscale(r10, c10));
  b01 = zadd(zcmul(r00, c01), zscale(r10, c11));
  b10 = zadd(zcmul(r01, c00), zscale(r11, c10));
  b11 = zadd(zcmul(r01, c01), zscale(r11, c11));
}

__device__ inline void rot_cols(const Rot& s, zc& zp, zc& zq) {
  const zc us = zmk(s.ur, s.ui);
  const zc s00 = zscale(s.c, us), s01 = zscale(s.s, us);
  const zc np = zadd(zmul(zp, s00), zscale(-s.s, zq));
  const zc nq = zadd(zmul(zp, s01), zscale(s.c, zq));
  zp = np;
  zq = nq;
}

constexpr int JACOBI_ZLDS_MAX = 64;  // G and Z both in LDS up to this size

__global__ void __launch_bounds__(1024) k_jacobi_small(const zc* G, int64_t ldg, int k, double* w, zc* Zout, int64_t ldz,
                                                      zc* Zg, double tau2, int* sweeps_out) {
  extern __shared__ zc Gs[];  // k x k, column-major ld k; then Z when k <= JACOBI_ZLDS_MAX
  __shared__ double red[16];
  __shared__ Rot prm[JACOBI_LDS_MAX / 2 + 1];
  __shared__ int pidx[JACOBI_LDS_MAX / 2 + 1], qidx[JACOBI_LDS_MAX / 2 + 1];
  __shared__ int rotated;
  zc* Z = (k <= JACOBI_ZLDS_MAX) ? Gs + k * k : Zg;
  const int tid = threadIdx.x;
  const int K2 = k + (k & 1), half = K2 / 2;
  const int nblk = half * (half + 1) / 2;
  double f = 0.0;
  for (int e = tid; e < k * k; e += blockDim.x) {
    const int i = e % k, j = e / k;
    zc v = G[i + (int64_t)j * ldg];
    if (i == j) v.y = 0.0;
    Gs[e] = v;
    Z[e] = zmk(i == j ? 1.0 : 0.0, 0.0);
    f += zabs2(v);
  }
  const double fro2 = block_sum(f, red);
  const double skip2 = fmax(1e-36 * fro2, tau2);
  int sweep = 0;
  for (; sweep < 100; sweep++) {
    double o = 0.0;
    for (int e = tid; e < k * k; e += blockDim.x)
      if (e % k != e / k) o += zabs2(Gs[e]);
    const double off2 = block_sum(o, red);
    if (off2 <= 1e-32 * fro2 || off2 == 0.0) break;
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < K2 - 1; r++) {
      if (tid < half) {
        int64_t p, q;
        round_pair(K2, r, tid, p, q);
        pidx[tid] = (int)p;
        qidx[tid] = (int)q;
        Rot R;
        if (q >= k) {
          R.c = 1.0; R.s = 0.0; R.ur = 1.0; R.ui = 0.0; R.tg = 0.0; R.active = 0;
        } else {
          R = make_rot(Gs[p + p * k], Gs[q + q * k], Gs[p + q * k], skip2);
          if (R.active) rotated = 1;
        }
        prm[tid] = R;
      }
      __syncthreads();
      // 2x2 blocks of pair rows rt >= pair columns st, mirrored (G Hermitian)
      for (int e = tid; e < nblk; e += blockDim.x) {
        int rt = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
        while (rt * (rt + 1) / 2 > e) rt--;
        while ((rt + 1) * (rt + 2) / 2 <= e) rt++;
        const int st = e - rt * (rt + 1) / 2;
        const Rot& Rr = prm[rt];
        const Rot& Rs = prm[st];
        if (!Rr.active && !Rs.active) continue;
        const int pr = pidx[rt], qr = qidx[rt], ps = pidx[st], qs = qidx[st];
        const bool qrv = qr < k, qsv = qs < k;
        zc b00 = Gs[pr + ps * k];
        zc b01 = qsv ? Gs[pr + qs * k] : zmk(0.0, 0.0);
        zc b10 = qrv ? Gs[qr + ps * k] : zmk(0.0, 0.0);
        zc b11 = (qrv && qsv) ? Gs[qr + qs * k] : zmk(0.0, 0.0);
        if (rt == st) {
          const double app = b00.x, aqq = b11.x;
          b00 = zmk(app - Rr.tg, 0.0);
          b11 = zmk(aqq + Rr.tg, 0.0);
          b01 = zmk(0.0, 0.0);
          b10 = zmk(0.0, 0.0);
        } else {
          rot_block(Rr, Rs, b00, b01, b10, b11);
        }
        Gs[pr + ps * k] = b00;
        if (qsv) Gs[pr + qs * k] = b01;
        if (qrv) Gs[qr + ps * k] = b10;
        if (qrv && qsv) Gs[qr + qs * k] = b11;
        if (rt != st) {
          Gs[ps + pr * k] = zconj(b00);
          if (qsv) Gs[qs + pr * k] = zconj(b01);
          if (qrv) Gs[ps + qr * k] = zconj(b10);
          if (qrv && qsv) Gs[qs + qr * k] = zconj(b11);
        }
      }
      for (int e = tid; e < k * half; e += blockDim.x) {
        const int i = e % k, st = e / k;
        const Rot& Rs = prm[st];
        if (!Rs.active) continue;
        const int ps = pidx[st], qs = qidx[st];
        zc zp = Z[i + ps * k], zq = Z[i + qs * k];
        rot_cols(Rs, zp, zq);
        Z[i + ps * k] = zp;
        Z[i + qs * k] = zq;
      }
      __syncthreads();
    }
    if (!rotated) break;
  }
  // stable ascending sort of the diagonal, columns of Z permuted alike
  for (int i = tid; i < k; i += blockDim.x) {
    const double di = Gs[i + i * k].x;
    int rank = 0;
    for (int j = 0; j < k; j++) {
      const double dj = Gs[j + j * k].x;
      if (dj < di || (dj == di && j < i)) rank++;
    }
    w[rank] = di;
    for (int r = 0; r < k; r++) Zout[r + (int64_t)rank * ldz] = Z[r + i * k];
  }
  if (tid == 0 && sweeps_out) *sweeps_out = sweep;
}

__global__ void k_jacobi_init(const zc* G, int64_t ldg, int64_t k, zc* G0, zc* Z0) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * k) return;
  const int64_t i = e % k, j = e / k;
  zc v = G[i + j * ldg];
  if (i == j) v.y = 0.0;
  G0[e] = v;
  Z0[e] = zmk(i == j ? 1.0 : 0.0, 0.0);
}

// ---- block sweeps: cyclic Jacobi in a block ordering ---------------------
// The indices are cut into blocks of BJB (the last one ragged; a phantom
// block makes the count even) and the blocks are paired round-robin.  In a
// round every pair of blocks (P, Q) is one 2 BJB x 2 BJB subproblem: one
// workgroup rotates its index pairs in LDS, accumulating the rotations in V
// -- in the first round of a sweep every index pair of P u Q once (which
// covers the pairs inside each block), in the other rounds the pairs across
// P and Q -- then every off-diagonal tile of G between two pairs' index sets
// is updated as V_s^H G(I_s, I_t) V_t and Z's columns as Z(:, I_t) V_t.
// Over the rounds every index pair (i, j) is rotated at least once (two
// blocks meet in exactly one round), which makes a round set one sweep of
// cyclic Jacobi in a block ordering; a sweep takes 2 launches per round
// instead of one launch per scalar round.
constexpr int BJB = 16;
constexpr int BJS = 2 * BJB;   // subproblem size
constexpr int BJL = BJS + 1;   // LDS leading dimension

// Global index of local index l (0 .. BJS-1) of the pair (P, Q); -1 outside
// the matrix (ragged last block, phantom block).
__device__ __forceinline__ int bjac_index(int64_t P, int64_t Q, int l, int64_t k, int64_t nb) {
  const int64_t blk = l < BJB ? P : Q;
  const int64_t g = blk * BJB + (l % BJB);
  return (blk < nb && g < k) ? (int)g : -1;
}

__global__ void __launch_bounds__(256) k_bjac_solve(zc* G, int64_t k, int64_t nb, int64_t NB2, int64_t round,
                                                    const double* fro2, double tau2, zc* V, int* rotated) {
  __shared__ zc S[BJS * BJL];   // the subproblem, column-major
  __shared__ zc Vs[BJS * BJL];  // its accumulated rotations
  __shared__ Rot prm[BJB];
  __shared__ int pidx[BJB], qidx[BJB], gi[BJS];
  __shared__ int any;
  const int tid = threadIdx.x;
  int64_t P, Q;
  round_pair(NB2, round, blockIdx.x, P, Q);
  if (tid < BJS) gi[tid] = bjac_index(P, Q, tid, k, nb);
  if (tid == 0) any = 0;
  __syncthreads();
  for (int e = tid; e < BJS * BJS; e += blockDim.x) {
    const int l = e % BJS, m = e / BJS;
    const int a = gi[l], b = gi[m];
    zc v = zmk(0.0, 0.0);
    if (a >= 0 && b >= 0) {
      v = G[a + (int64_t)b * k];
      if (l == m) v.y = 0.0;
    }
    S[l + m * BJL] = v;
    Vs[l + m * BJL] = zmk(l == m ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const double skip2 = fmax(1e-36 * fro2[0], tau2);
  constexpr int NBLK = BJB * (BJB + 1) / 2;
  // the first round of a sweep visits every index pair of P u Q (31
  // disjoint-pair rounds: the pairs inside a block are covered there);
  // the other rounds visit the pairs across P and Q only (16 rounds,
  // i in P with Q's (i + r) mod 16)
  const bool full = round == 0;
  const int inner = full ? BJS - 1 : BJB;
  for (int r = 0; r < inner; r++) {
    if (tid < BJB) {
      int64_t p, q;
      if (full) {
        round_pair(BJS, r, tid, p, q);
      } else {
        p = tid;
        q = BJB + (tid + r) % BJB;
      }
      pidx[tid] = (int)p;
      qidx[tid] = (int)q;
      Rot R;
      R.c = 1.0; R.s = 0.0; R.ur = 1.0; R.ui = 0.0; R.tg = 0.0; R.active = 0;
      if (gi[p] >= 0 && gi[q] >= 0) {
        R = make_rot(S[p + p * BJL], S[q + q * BJL], S[p + q * BJL], skip2);
        if (R.active) any = 1;
      }
      prm[tid] = R;
    }
    __syncthreads();
    // 2x2 blocks of pair rows rt >= pair columns st, mirrored (S Hermitian);
    // indices outside the matrix have zero rows and columns and inactive
    // rotations, so they stay decoupled
    for (int e = tid; e < NBLK; e += blockDim.x) {
      int rt = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
      while (rt * (rt + 1) / 2 > e) rt--;
      while ((rt + 1) * (rt + 2) / 2 <= e) rt++;
      const int st = e - rt * (rt + 1) / 2;
      const Rot& Rr = prm[rt];
      const Rot& Rs = prm[st];
      if (!Rr.active && !Rs.active) continue;
      const int pr = pidx[rt], qr = qidx[rt], ps = pidx[st], qs = qidx[st];
      zc b00 = S[pr + ps * BJL], b01 = S[pr + qs * BJL], b10 = S[qr + ps * BJL], b11 = S[qr + qs * BJL];
      if (rt == st) {
        const double app = b00.x, aqq = b11.x;
        b00 = zmk(app - Rr.tg, 0.0);
        b11 = zmk(aqq + Rr.tg, 0.0);
        b01 = zmk(0.0, 0.0);
        b10 = zmk(0.0, 0.0);
      } else {
        rot_block(Rr, Rs, b00, b01, b10, b11);
      }
      S[pr + ps * BJL] = b00;
      S[pr + qs * BJL] = b01;
      S[qr + ps * BJL] = b10;
      S[qr + qs * BJL] = b11;
      if (rt != st) {
        S[ps + pr * BJL] = zconj(b00);
        S[qs + pr * BJL] = zconj(b01);
        S[ps + qr * BJL] = zconj(b10);
        S[qs + qr * BJL] = zconj(b11);
      }
    }
    for (int e = tid; e < BJS * BJB; e += blockDim.x) {
      const int i = e % BJS, st = e / BJS;
      const Rot& Rs = prm[st];
      if (!Rs.active) continue;
      const int ps = pidx[st], qs = qidx[st];
      zc zp = Vs[i + ps * BJL], zq = Vs[i + qs * BJL];
      rot_cols(Rs, zp, zq);
      Vs[i + ps * BJL] = zp;
      Vs[i + qs * BJL] = zq;
    }
    __syncthreads();
  }
  // the pair's diagonal tile of G and its rotations out
  zc* Vo = V + (int64_t)blockIdx.x * BJS * BJS;
  for (int e = tid; e < BJS * BJS; e += blockDim.x) {
    const int l = e % BJS, m = e / BJS;
    const int a = gi[l], b = gi[m];
    if (a >= 0 && b >= 0) G[a + (int64_t)b * k] = S[l + m * BJL];
    Vo[e] = Vs[l + m * BJL];
  }
  if (tid == 0 && any) *rotated = 1;
}

// Workgroups [0, NP (NP - 1) / 2): tile (s, t), s > t, of G between pair s's
// and pair t's index sets, G(I_s, I_t) <- V_s^H G(I_s, I_t) V_t, and its
// mirror G(I_t, I_s) <- the conjugate transpose; then NP * ceil(k / BJS)
// workgroups: Z(rows, I_t) <- Z(rows, I_t) V_t.  Each workgroup reads and
// writes only its own tile (and the mirror, which no workgroup reads), so
// the update is in place.
__global__ void __launch_bounds__(256) k_bjac_update(zc* G, zc* Z, int64_t k, int64_t nb, int64_t NB2, int64_t round,
                                                     const zc* V) {
  static_assert(BJS * BJS % 256 == 0, "whole tiles per workgroup");
  constexpr int PER = BJS * BJS / 256;  // tile entries per thread
  __shared__ zc Ts[BJS * BJL];          // the tile, then G(I_s, I_t) V_t
  __shared__ zc Va[BJS * BJL];
  __shared__ zc Vb[BJS * BJL];
  __shared__ int ga[BJS], gb[BJS];
  const int tid = threadIdx.x;
  const int64_t NP = NB2 / 2;
  const int64_t ntile = NP * (NP - 1) / 2;
  const int64_t bid = blockIdx.x;
  if (bid < ntile) {
    int64_t s = (int64_t)((sqrt(8.0 * (double)bid + 1.0) + 1.0) * 0.5);
    while (s * (s - 1) / 2 > bid) s--;
    while ((s + 1) * s / 2 <= bid) s++;
    const int64_t t = bid - s * (s - 1) / 2;  // 0 <= t < s
    int64_t Ps, Qs, Pt, Qt;
    round_pair(NB2, round, s, Ps, Qs);
    round_pair(NB2, round, t, Pt, Qt);
    if (tid < BJS) {
      ga[tid] = bjac_index(Ps, Qs, tid, k, nb);
      gb[tid] = bjac_index(Pt, Qt, tid, k, nb);
    }
    __syncthreads();
    const zc* V_s = V + s * BJS * BJS;
    const zc* V_t = V + t * BJS * BJS;
    for (int e = tid; e < BJS * BJS; e += blockDim.x) {
      const int l = e % BJS, m = e / BJS;
      const int a = ga[l], b = gb[m];
      Ts[l + m * BJL] = (a >= 0 && b >= 0) ? G[a + (int64_t)b * k] : zmk(0.0, 0.0);
      Va[l + m * BJL] = V_s[e];
      Vb[l + m * BJL] = V_t[e];
    }
    __syncthreads();
    zc w[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const int e = tid + 256 * u, l = e % BJS, m = e / BJS;
      zc acc = zmk(0.0, 0.0);
#pragma unroll 8
      for (int j = 0; j < BJS; j++) acc = zadd(acc, zmul(Ts[l + j * BJL], Vb[j + m * BJL]));
      w[u] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const int e = tid + 256 * u;
      Ts[e % BJS + (e / BJS) * BJL] = w[u];
    }
    __syncthreads();
    for (int e = tid; e < BJS * BJS; e += blockDim.x) {
      const int l = e % BJS, m = e / BJS;
      const int a = ga[l], b = gb[m];
      zc acc = zmk(0.0, 0.0);
#pragma unroll 8
      for (int j = 0; j < BJS; j++) acc = zadd(acc, zcmul(Va[j + l * BJL], Ts[j + m * BJL]));
      if (a >= 0 && b >= 0) {
        G[a + (int64_t)b * k] = acc;
        G[b + (int64_t)a * k] = zconj(acc);
      }
    }
    return;
  }
  const int64_t zb = bid - ntile;
  const int64_t t = zb % NP, r0 = (zb / NP) * BJS;
  int64_t Pt, Qt;
  round_pair(NB2, round, t, Pt, Qt);
  if (tid < BJS) gb[tid] = bjac_index(Pt, Qt, tid, k, nb);
  __syncthreads();
  const zc* V_t = V + t * BJS * BJS;
  for (int e = tid; e < BJS * BJS; e += blockDim.x) {
    const int i = e % BJS, m = e / BJS;
    const int b = gb[m];
    Ts[i + m * BJL] = (r0 + i < k && b >= 0) ? Z[(r0 + i) + (int64_t)b * k] : zmk(0.0, 0.0);
    Vb[i + m * BJL] = V_t[e];
  }
  __syncthreads();
  for (int e = tid; e < BJS * BJS; e += blockDim.x) {
    const int i = e % BJS, m = e / BJS;
    const int b = gb[m];
    zc acc = zmk(0.0, 0.0);
#pragma unroll 8
    for (int j = 0; j < BJS; j++) acc = zadd(acc, zmul(Ts[i + j * BJL], Vb[j + m * BJL]));
    if (r0 + i < k && b >= 0) Z[(r0 + i) + (int64_t)b * k] = acc;
  }
}

// ---- sparse sweeps: only the pairs whose coupling is significant ----------
// counts[j] = #{ i > j : |G(i, j)|^2 > thr_factor * fro2 }
// Selected pairs (i, j), i > j, per column j: |G_ij|^2 above
// max(thr_factor ||G||_F^2, tau^2) and, with ratio > 0, |G_ij| above ratio
// times |G_ii - G_jj| (the couplings that keep the matrix from being nearly
// diagonal).
__device__ __forceinline__ bool jacobi_selected(const zc* G, int64_t k, int64_t i, int64_t j, double thr, double ratio) {
  const double g2 = zabs2(G[i + j * k]);
  if (!(g2 > thr)) return false;
  if (ratio <= 0.0) return true;
  const double d = G[i + i * k].x - G[j + j * k].x;
  return g2 > ratio * ratio * d * d;
}

// One wave (64 threads) per column j walks rows i > j in chunks of 64;
// ballots give each selected pair its rank, so the list keeps the
// ascending row order within a column.
__global__ void __launch_bounds__(64) k_jacobi_count(const zc* G, int64_t k, const double* fro2, double thr_factor,
                                                     double tau2, double ratio, int* counts) {
  const int64_t j = blockIdx.x;
  const int lane = threadIdx.x;
  const double thr = fmax(thr_factor * fro2[0], tau2);
  int c = 0;
  for (int64_t i0 = j + 1; i0 < k; i0 += 64) {
    const int64_t i = i0 + lane;
    const bool sel = i < k && jacobi_selected(G, k, i, j, thr, ratio);
    c += __popcll(__ballot(sel));
  }
  if (lane == 0) counts[j] = c;
}

// pairs (j, i), i > j, of column j at offsets[j] (ascending i)
__global__ void __launch_bounds__(64) k_jacobi_list(const zc* G, int64_t k, const double* fro2, double thr_factor,
                                                    double tau2, double ratio, const int* offsets, int* pairs) {
  const int64_t j = blockIdx.x;
  const int lane = threadIdx.x;
  const double thr = fmax(thr_factor * fro2[0], tau2);
  const unsigned long long below = (1ull << lane) - 1ull;
  int o = offsets[j];
  for (int64_t i0 = j + 1; i0 < k; i0 += 64) {
    const int64_t i = i0 + lane;
    const bool sel = i < k && jacobi_selected(G, k, i, j, thr, ratio);
    const unsigned long long m = __ballot(sel);
    if (sel) {
      const int pos = o + __popcll(m & below);
      pairs[2 * pos] = (int)j;
      pairs[2 * pos + 1] = (int)i;
    }
    o += __popcll(m);
  }
}

// rotation parameters of one round's disjoint pairs (read before any update)
__global__ void k_jacobi_params(const zc* G, int64_t k, const int* pairs, int np, const double* fro2, double tau2, Rot* prm,
                                int* rotated) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= np) return;
  const int64_t p = pairs[2 * a], q = pairs[2 * a + 1];
  const Rot R = make_rot(G[p + p * k], G[q + q * k], G[p + q * k], fmax(1e-36 * fro2[0], tau2));
  if (R.active) *rotated = 1;
  prm[a] = R;
}

// In-place application of one round: work item (a, j) updates the block of
// pair a's rows with index j's group (j's pair when j is its first member
// and that pair is not after a; j alone when unpaired) and its mirror; the
// second half of the items rotates Z's columns.
__global__ void k_jacobi_apply(zc* G, zc* Z, int64_t k, const int* pairs, int np, const int* pairof, const Rot* prm) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)np * k) {
    const int a = (int)(e / k);
    const int64_t j = e % k;
    const Rot Ra = prm[a];
    const int64_t pa = pairs[2 * a], qa = pairs[2 * a + 1];
    const int b = pairof[j];
    if (b < 0) {
      // unpaired column j: rows (pa, qa) rotate, column j does not
      if (!Ra.active) return;
      Rot I;
      I.c = 1.0; I.s = 0.0; I.ur = 1.0; I.ui = 0.0; I.tg = 0.0; I.active = 0;
      zc b00 = G[pa + j * k], b01 = zmk(0.0, 0.0), b10 = G[qa + j * k], b11 = zmk(0.0, 0.0);
      rot_block(Ra, I, b00, b01, b10, b11);
      G[pa + j * k] = b00;
      G[qa + j * k] = b10;
      G[j + pa * k] = zconj(b00);
      G[j + qa * k] = zconj(b10);
      return;
    }
    const int64_t pb = pairs[2 * b], qb = pairs[2 * b + 1];
    if (j != pb || b > a) return;
    const Rot Rb = prm[b];
    if (!Ra.active && !Rb.active) return;
    zc b00 = G[pa + pb * k], b01 = G[pa + qb * k], b10 = G[qa + pb * k], b11 = G[qa + qb * k];
    if (a == b) {
      const double app = b00.x, aqq = b11.x;
      G[pa + pa * k] = zmk(app - Ra.tg, 0.0);
      G[qa + qa * k] = zmk(aqq + Ra.tg, 0.0);
      G[pa + qa * k] = zmk(0.0, 0.0);
      G[qa + pa * k] = zmk(0.0, 0.0);
      return;
    }
    rot_block(Ra, Rb, b00, b01, b10, b11);
    G[pa + pb * k] = b00;
    G[pa + qb * k] = b01;
    G[qa + pb * k] = b10;
    G[qa + qb * k] = b11;
    G[pb + pa * k] = zconj(b00);
    G[qb + pa * k] = zconj(b01);
    G[pb + qa * k] = zconj(b10);
    G[qb + qa * k] = zconj(b11);
    return;
  }
  const int64_t e2 = e - (int64_t)np * k;
  if (e2 >= (int64_t)np * k) return;
  const int a = (int)(e2 / k);
  const int64_t i = e2 % k;
  const Rot Ra = prm[a];
  if (!Ra.active) return;
  const int64_t pa = pairs[2 * a], qa = pairs[2 * a + 1];
  zc zp = Z[i + pa * k], zq = Z[i + qa * k];
  rot_cols(Ra, zp, zq);
  Z[i + pa * k] = zp;
  Z[i + qa * k] = zq;
}

__global__ void k_jacobi_norms_part(const zc* G, int64_t k, double* part) {
  __shared__ double red[16];
  double off = 0.0, all = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < k * k; e += (int64_t)gridDim.x * blockDim.x) {
    const double a = zabs2(G[e]);
    all += a;
    if (e % k != e / k) off += a;
  }
  off = block_sum(off, red);
  all = block_sum(all, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = off;
    part[2 * blockIdx.x + 1] = all;
  }
}

__global__ void k_jacobi_norms_final(const double* part, int nb, double* out) {
  if (threadIdx.x == 0) {
    double off = 0.0, all = 0.0;
    for (int b = 0; b < nb; b++) {
      off += part[2 * b];
      all += part[2 * b + 1];
    }
    out[0] = off;
    out[1] = all;
  }
}

__global__ void k_jacobi_rank(const zc* G, int64_t k, int* rank, double* w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const double di = G[i + i * k].x;
  int r = 0;
  for (int64_t j = 0; j < k; j++) {
    const double dj = G[j + j * k].x;
    if (dj < di || (dj == di && j < i)) r++;
  }
  rank[i] = r;
  w[r] = di;
}

__global__ void k_jacobi_permute(const zc* Z, int64_t k, const int* rank, zc* Zout, int64_t ldz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= k * k) return;
  const int64_t r = e % k, i = e / k;
  Zout[r + (int64_t)rank[i] * ldz] = Z[e];
}

// --------------------------------------------------------------------------
// Iterative refinement of the eigenvectors of a nearly diagonal Hermitian G
// (the projected matrix once the block is close to invariant).  X holds
// approximate eigenvectors; with S = X^H G X, P = X^H X, R = I - P and the
// Rayleigh quotients lam_i = Re S_ii / P_ii, one step sets
//   E_ij = (S_ij + lam_j R_ij) / (lam_j - lam_i)   for coupled pairs,
//   E_ij = R_ij / 2                                for pairs whose coupling is
//                                                  below tau (and i = j),
//   X <- X + X E.
// (Ogita and Aishima's refinement for symmetric eigenproblems, with a
// threshold instead of their cluster test.)  The decision for a pair uses
// max(|S_ij + lam_j R_ij|, |S_ij + lam_i R_ij|), which is the same for (i, j)
// and (j, i) when S and P are exactly Hermitian, so E_ij + conj(E_ji) = R_ij
// and the orthogonality error is corrected together with the coupling.
// corr (bit pattern of a non-negative double) receives max |E_ij| over i != j,
// +inf for a non-finite value.
// --------------------------------------------------------------------------
// (S, P are read as their Hermitian parts (M + M^H)/2: the products that
// form them are Hermitian only up to rounding.)  corr_next (nullable) is
// zeroed for the next step's maximum.
__global__ void k_refine_coeffs(const zc* S, const zc* P, int64_t k, double tau, zc* E, zc* Xout, double* lam,
                                unsigned long long* corr, unsigned long long* corr_next) {
  __shared__ double red[NT / 64];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (corr_next && e == 0) *corr_next = 0ull;
  double c = 0.0;
  if (e < k * k) {
    const int64_t i = e % k, j = e / k;
    const double pii = P ? P[i + i * k].x : 1.0, pjj = P ? P[j + j * k].x : 1.0;
    const double li = S[i + i * k].x / pii, lj = S[j + j * k].x / pjj;
    zc ev;
    if (i == j) {
      ev = zmk(0.5 * (1.0 - pii), 0.0);
      if (lam) lam[i] = li;
    } else {
      const int64_t et = j + i * k;
      zc r = zmk(0.0, 0.0);
      if (P) {
        const zc a = P[e], b = P[et];
        r = zmk(-(0.5 * (a.x + b.x)), -(0.5 * (a.y - b.y)));
      }
      const zc s0 = S[e], s1 = S[et];
      const zc sij = zmk(0.5 * (s0.x + s1.x), 0.5 * (s0.y - s1.y));
      const zc n1 = zadd(sij, zscale(lj, r)), n2 = zadd(sij, zscale(li, r));
      const double m2 = fmax(zabs2(n1), zabs2(n2));
      if (m2 > tau * tau) ev = zscale(1.0 / (lj - li), n1);
      else ev = zscale(0.5, r);
      c = sqrt(zabs2(ev));
      if (!(c <= 1.7976931348623157e308)) c = INFINITY;
    }
    E[e] = ev;
    if (Xout) Xout[e] = i == j ? zmk(1.0 + ev.x, ev.y) : ev;
  }
  // block max (non-negative values: max of the bit patterns)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c = fmax(c, __shfl_xor(c, off, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); q++) m = fmax(m, red[q]);
    atomicMax(corr, (unsigned long long)__double_as_longlong(m));
  }
}

// rank of each value (ties by index) and the sorted values
__global__ void k_rank_values(const double* lam, int64_t k, int* rank, double* w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const double di = lam[i];
  int r = 0;
  for (int64_t j = 0; j < k; j++) {
    const double dj = lam[j];
    if (dj < di || (dj == di && j < i)) r++;
  }
  rank[i] = r;
  w[r] = di;
}

// --------------------------------------------------------------------------
// Lanczos pieces
// --------------------------------------------------------------------------
constexpr int MV_SPLITS = 32;

__global__ void k_gemv_part(const zc* A, int64_t lda, int64_t n, const zc* x, zc* part) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  const int64_t cs = cdiv(n, MV_SPLITS);
  const int64_t c0 = s * cs, c1 = min(n, c0 + cs);
  if (i >= n) return;
  zc acc = zmk(0.0, 0.0);
  for (int64_t c = c0; c < c1; c++) acc = zadd(acc, zmul(A[i + c * lda], x[c]));
  part[(int64_t)s * n + i] = acc;
}

__global__ void k_gemv_reduce(const zc* part, int64_t n, zc* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  zc acc = zmk(0.0, 0.0);
  for (int s = 0; s < MV_SPLITS; s++) acc = zadd(acc, part[(int64_t)s * n + i]);
  y[i] = acc;
}

__global__ void k_multi_dot(const zc* V, int64_t ldv, int64_t n, const zc* w, zc* out) {
  __shared__ double red[16];
  const int64_t p = blockIdx.x;
  double re = 0.0, im = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const zc t = zcmul(V[i + p * ldv], w[i]);
    re += t.x;
    im += t.y;
  }
  re = block_sum(re, red);
  im = block_sum(im, red);
  if (threadIdx.x == 0) out[p] = zmk(re, im);
}

__global__ void k_sub_combination(const zc* V, int64_t ldv, int64_t n, int64_t cnt, const zc* h, zc* w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  zc acc = w[i];
  for (int64_t p = 0; p < cnt; p++) acc = zsub(acc, zmul(V[i + p * ldv], h[p]));
  w[i] = acc;
}

__global__ void k_three_term(zc* w, const zc* V, int64_t ldv, int64_t n, int64_t j, double* alpha, const double* beta,
                             const zc* h) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double a = h[0].x;
  if (i == 0) alpha[j] = a;
  if (i >= n) return;
  zc acc = zsub(w[i], zscale(a, V[i + j * ldv]));
  if (j > 0) acc = zsub(acc, zscale(beta[j], V[i + (j - 1) * ldv]));
  w[i] = acc;
}

__global__ void k_norm(const zc* w, int64_t n, double* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += zabs2(w[i]);
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[0] = sqrt(s);
}

__global__ void k_scale_inv(const zc* w, int64_t n, const double* nrm, zc* v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double b = nrm[0];
  v[i] = b > 0.0 ? zscale(1.0 / b, w[i]) : zmk(0.0, 0.0);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define LAUNCH(kern, grid, block, shm, st, ...)                          \
  do {                                                                  \
    hipLaunchKernelGGL(kern, grid, block, shm, st, __VA_ARGS__);        \
    CHFSI_CHECK_LAUNCH();                                               \
  } while (0)

void random_block(uint64_t seed, uint32_t stream, int64_t n, int64_t k, int64_t col0, zc* Y, int64_t ldy, hipStream_t st) {
  if (n * k == 0) return;
  LAUNCH(k_random_block, grid1(n * k), dim3(NT), 0, st, seed, stream, n, k, col0, Y, ldy);
}

void philox_raw(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count, hipStream_t st) {
  if (count == 0) return;
  LAUNCH(k_philox_raw, grid1(count), dim3(NT), 0, st, ctr, key, out, count);
}

void fill_i32(int* p, int64_t count, int v, hipStream_t st) {
  if (count == 0) return;
  LAUNCH(k_fill_i32, grid1(count), dim3(NT), 0, st, p, count, v);
}

void copy2d(const zc* src, int64_t lds, zc* dst, int64_t ldd, int64_t m, int64_t n, hipStream_t st) {
  if (m * n == 0) return;
  LAUNCH(k_copy2d, grid1(m * n), dim3(NT), 0, st, src, lds, dst, ldd, m, n);
}

void lincomb2d(double a, const zc* X, int64_t ldx, double b, const zc* Y, int64_t ldy, zc* out, int64_t ldo, int64_t m,
               int64_t n, hipStream_t st) {
  if (m * n == 0) return;
  LAUNCH(k_lincomb2d, grid1(m * n), dim3(NT), 0, st, a, X, ldx, b, Y, ldy, out, ldo, m, n);
}

void to_f32(const zc* src, int64_t lds, cc* dst, int64_t ldd, int64_t m, int64_t n, hipStream_t st) {
  if (m * n == 0) return;
  LAUNCH(k_z2c, grid1(m * n), dim3(NT), 0, st, src, lds, dst, ldd, m, n);
}

void to_f64(const cc* src, int64_t lds, zc* dst, int64_t ldd, int64_t m, int64_t n, hipStream_t st) {
  if (m * n == 0) return;
  LAUNCH(k_c2z, grid1(m * n), dim3(NT), 0, st, src, lds, dst, ldd, m, n);
}

void ritz_forcing(const zc* Y0, int64_t ldy, const zc* AY0, int64_t lday, const double* mu, double alpha0, cc* R,
                  int64_t ldr, cc* D1, int64_t ldd, double* scale, int64_t m, int64_t n, hipStream_t st) {
  if (m * n == 0) return;
  LAUNCH(k_ritz_forcing, dim3((unsigned)n), dim3(256), 0, st, Y0, ldy, AY0, lday, mu, alpha0, R, ldr, D1, ldd, scale, m);
}

void ritz_combine(const zc* Y0, int64_t ldy, const double* t, const double* scale, const cc* D, int64_t ldd, zc* F,
                  int64_t ldf, int64_t m, int64_t n, hipStream_t st) {
  if (m * n == 0) return;
  LAUNCH(k_ritz_combine, grid1(m * n), dim3(NT), 0, st, Y0, ldy, t, scale, D, ldd, F, ldf, m, n);
}

void set_identity(zc* Y, int64_t ldy, int64_t m, int64_t n, hipStream_t st) {
  if (m * n == 0) return;
  LAUNCH(k_set_identity, grid1(m * n), dim3(NT), 0, st, Y, ldy, m, n);
}

void zero_strict_upper(zc* A, int64_t lda, int64_t n, hipStream_t st) {
  LAUNCH(k_zero_strict_upper, grid1(n * n), dim3(NT), 0, st, A, lda, n);
}

void hermitian_from_lower(zc* A, int64_t lda, int64_t n, hipStream_t st) {
  LAUNCH(k_hermitian_from_lower, grid1(n * n), dim3(NT), 0, st, A, lda, n);
}

void residual_block(const zc* W, int64_t ldw, const zc* Y, int64_t ldy, const double* mu, zc* R, int64_t ldr, int64_t n,
                    int64_t k, hipStream_t st) {
  if (n * k == 0) return;
  LAUNCH(k_residual, grid1(n * k), dim3(NT), 0, st, W, ldw, Y, ldy, mu, R, ldr, n, k);
}

void column_norms(const zc* R, int64_t ldr, int64_t n, int64_t k, double* out, hipStream_t st) {
  if (k == 0) return;
  LAUNCH(k_column_norms, dim3((unsigned)k), dim3(NT), 0, st, R, ldr, n, out);
}

void diag_ratio(const zc* L, int64_t ld, int64_t k, double* out, hipStream_t st) {
  LAUNCH(k_diag_ratio, dim3(1), dim3(256), 0, st, L, ld, k, out);
}


void chol_diag(const zc* W, int64_t ldw, zc* L, int64_t ldl, zc* Linv, int64_t ldi, int64_t j0, int64_t nb, int* info,
               hipStream_t st) {
  static std::once_flag attr;
  const size_t shm = (size_t)(2 * CNB * CLD + CNB * CNB / 4) * sizeof(zc);
  std::call_once(attr, [&] {
    CHFSI_HIP(hipFuncSetAttribute((const void*)k_chol_diag, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  });
  if (nb < 1 || nb > CNB) throw Error(ST_EINVAL, "chol_diag: block size out of range");
  LAUNCH(k_chol_diag, dim3(1), dim3(CNT), shm, st, W, ldw, L, ldl, Linv, ldi, j0, (int)nb, info);
}

void hh_panel_setup(HHPanel& p) {
  const int64_t rows = p.n - p.j0;
  int64_t nb = std::min<int64_t>(cdiv(rows, 256), 240);
  if (nb < 1) nb = 1;
  p.rows_per_blk = 256 * cdiv(cdiv(rows, nb), 256);
  p.nblk = (int)cdiv(rows, p.rows_per_blk);
  if (p.nblk < 1) p.nblk = 1;
}

void hh_first_partials(const HHPanel& p, hipStream_t st) {
  LAUNCH(k_hh_first, dim3((unsigned)p.nblk), dim3(256), 0, st, p);
}

void hh_column(const HHPanel& p, int64_t j, hipStream_t st) {
  LAUNCH(k_hh_column, dim3((unsigned)p.nblk), dim3(256), 0, st, p, j);
}

void hh_extract_v(const zc* F, int64_t ldf, int64_t n, int64_t j0, int64_t j1, zc* Vp, int64_t ldv, hipStream_t st) {
  const int64_t tot = (n - j0) * (j1 - j0);
  if (tot == 0) return;
  LAUNCH(k_hh_extract_v, grid1(tot), dim3(NT), 0, st, F, ldf, n, j0, j1, Vp, ldv);
}

void hh_build_t(const zc* gram, const zc* tau, int64_t cnt, zc* T, hipStream_t st) {
  LAUNCH(k_hh_build_t, dim3(1), dim3(64), 0, st, gram, tau, cnt, T);
}

void jacobi_small(const zc* G, int64_t ldg, int64_t k, double* w, zc* Z, int64_t ldz, zc* Ztmp, int* sweeps_out,
                  hipStream_t st, double tau) {
  if (k < 1 || k > JACOBI_LDS_MAX) throw Error(ST_EINVAL, "jacobi_small: size out of range");
  static std::once_flag attr;
  const size_t shm = (size_t)JACOBI_LDS_MAX * JACOBI_LDS_MAX * sizeof(zc);
  std::call_once(attr, [&] {
    CHFSI_HIP(hipFuncSetAttribute((const void*)k_jacobi_small, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  });
  const size_t dyn = (size_t)k * k * sizeof(zc) * (k <= JACOBI_ZLDS_MAX ? 2 : 1);
  LAUNCH(k_jacobi_small, dim3(1), dim3(1024), dyn, st, G, ldg, (int)k, w, Z, ldz, Ztmp, tau * tau, sweeps_out);
}

void jacobi_init(const zc* G, int64_t ldg, int64_t k, zc* G0, zc* Z0, hipStream_t st) {
  LAUNCH(k_jacobi_init, grid1(k * k), dim3(NT), 0, st, G, ldg, k, G0, Z0);
}

size_t block_jacobi_v_bytes(int64_t k) {
  const int64_t nb = cdiv(k, (int64_t)BJB), NB2 = nb + (nb & 1);
  return (size_t)(NB2 / 2) * BJS * BJS * sizeof(zc);
}

void block_jacobi_round(zc* G, zc* Z, int64_t k, int64_t round, const double* fro2, double tau, zc* V, int* rotated,
                        hipStream_t st) {
  const int64_t nb = cdiv(k, (int64_t)BJB), NB2 = nb + (nb & 1), NP = NB2 / 2;
  if (k < 1 || round < 0 || round >= NB2 - 1) throw Error(ST_EINVAL, "block_jacobi_round: bad size or round");
  LAUNCH(k_bjac_solve, dim3((unsigned)NP), dim3(256), 0, st, G, k, nb, NB2, round, fro2, tau * tau, V, rotated);
  const int64_t grid = NP * (NP - 1) / 2 + NP * cdiv(k, (int64_t)BJS);
  LAUNCH(k_bjac_update, dim3((unsigned)grid), dim3(256), 0, st, G, Z, k, nb, NB2, round, (const zc*)V);
}

int64_t block_jacobi_rounds(int64_t k) {
  const int64_t nb = cdiv(k, (int64_t)BJB);
  return nb + (nb & 1) - 1;
}

void jacobi_count(const zc* G, int64_t k, const double* fro2, double thr_factor, double tau, double ratio, int* counts,
                  hipStream_t st) {
  LAUNCH(k_jacobi_count, dim3((unsigned)k), dim3(64), 0, st, G, k, fro2, thr_factor, tau * tau, ratio, counts);
}

void jacobi_list(const zc* G, int64_t k, const double* fro2, double thr_factor, double tau, double ratio,
                 const int* offsets, int* pairs, hipStream_t st) {
  LAUNCH(k_jacobi_list, dim3((unsigned)k), dim3(64), 0, st, G, k, fro2, thr_factor, tau * tau, ratio, offsets, pairs);
}

void jacobi_sparse_round(zc* G, zc* Z, int64_t k, const int* pairs, int np, const int* pairof, void* prm_scratch,
                         const double* fro2, double tau, int* rotated, hipStream_t st) {
  if (np == 0) return;
  Rot* prm = static_cast<Rot*>(prm_scratch);
  LAUNCH(k_jacobi_params, grid1(np), dim3(NT), 0, st, G, k, pairs, np, fro2, tau * tau, prm, rotated);
  LAUNCH(k_jacobi_apply, grid1(2 * (int64_t)np * k), dim3(NT), 0, st, G, Z, k, pairs, np, pairof, prm);
}

size_t jacobi_rot_bytes() { return sizeof(Rot); }

void jacobi_norms(const zc* G, int64_t k, double* part, double* out, hipStream_t st) {
  const int nb = (int)std::min<int64_t>(256, std::max<int64_t>(1, cdiv(k * k, 1024)));
  LAUNCH(k_jacobi_norms_part, dim3(nb), dim3(NT), 0, st, G, k, part);
  LAUNCH(k_jacobi_norms_final, dim3(1), dim3(64), 0, st, part, nb, out);
}

void jacobi_sort(const zc* G, const zc* Z, int64_t k, double* w, int* rank, zc* Zout, int64_t ldz, hipStream_t st) {
  LAUNCH(k_jacobi_rank, grid1(k), dim3(NT), 0, st, G, k, rank, w);
  LAUNCH(k_jacobi_permute, grid1(k * k), dim3(NT), 0, st, Z, k, rank, Zout, ldz);
}

void refine_coeffs(const zc* S, const zc* P, int64_t k, double tau, zc* E, zc* Xout, double* lam,
                   unsigned long long* corr, unsigned long long* corr_next, hipStream_t st) {
  LAUNCH(k_refine_coeffs, grid1(k * k), dim3(NT), 0, st, S, P, k, tau, E, Xout, lam, corr, corr_next);
}

void sort_by_values(const double* lam, const zc* Z, int64_t k, double* w, int* rank, zc* Zout, int64_t ldz,
                    hipStream_t st) {
  LAUNCH(k_rank_values, grid1(k), dim3(NT), 0, st, lam, k, rank, w);
  LAUNCH(k_jacobi_permute, grid1(k * k), dim3(NT), 0, st, Z, k, rank, Zout, ldz);
}

void zgemv(const zc* A, int64_t lda, int64_t n, const zc* x, zc* y, zc* part, hipStream_t st) {
  LAUNCH(k_gemv_part, dim3((unsigned)cdiv(n, NT), MV_SPLITS), dim3(NT), 0, st, A, lda, n, x, part);
  LAUNCH(k_gemv_reduce, grid1(n), dim3(NT), 0, st, part, n, y);
}

void multi_dot(const zc* V, int64_t ldv, int64_t n, int64_t cnt, const zc* w, zc* out, hipStream_t st) {
  if (cnt == 0) return;
  LAUNCH(k_multi_dot, dim3((unsigned)cnt), dim3(NT), 0, st, V, ldv, n, w, out);
}

void sub_combination(const zc* V, int64_t ldv, int64_t n, int64_t cnt, const zc* h, zc* w, hipStream_t st) {
  if (cnt == 0) return;
  LAUNCH(k_sub_combination, grid1(n), dim3(NT), 0, st, V, ldv, n, cnt, h, w);
}

void lanczos_three_term(zc* w, const zc* V, int64_t ldv, int64_t n, int64_t j, double* alpha, const double* beta,
                        const zc* h, hipStream_t st) {
  LAUNCH(k_three_term, grid1(n), dim3(NT), 0, st, w, V, ldv, n, j, alpha, beta, h);
}

void normalize(const zc* w, int64_t n, zc* v, double* beta_out, hipStream_t st) {
  LAUNCH(k_norm, dim3(1), dim3(1024), 0, st, w, n, beta_out);
  LAUNCH(k_scale_inv, grid1(n), dim3(NT), 0, st, w, n, beta_out, v);
}

}  // namespace chfsi
