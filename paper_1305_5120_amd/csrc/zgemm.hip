// Complex FP64 GEMM on gfx950 matrix cores with a fused three-term epilogue.
//
//   out = alpha * op(A) op(B) + beta * X + gamma * Z      (alpha, beta, gamma real)
//
// This is the Chebyshev filter step of Algorithm 1 (eq. (3), scaled and
// shifted): with op = N, X = Y_i and Z = Y_{i-1}, one launch computes
// Y_{i+1} = alpha A Y_i + beta Y_i + gamma Y_{i-1} and writes it over Y_{i-1},
// so every degree step reads A, Y_i, Y_{i-1} and writes Y_{i+1} once.  The
// same kernel (other op / flag combinations) serves every other dense product
// of the solver (Cholesky updates, triangular inverse, reduction to standard
// form, Householder block updates, Rayleigh-Ritz, back-transform).
//
// Design (CDNA4):
//   * 256 threads = 4 waves in a 2x2 arrangement; a workgroup owns a BM x BN
//     complex output tile, each wave (BM/2) x (BN/2) of it as 16x16 blocks;
//   * complex products as four real v_mfma_f64_16x16x4f64 per 16x16x4 block
//     into separate real / imaginary accumulators;
//   * K is walked in slabs of BK complex elements staged through LDS, double
//     buffered: the next slab's global loads are in flight while the current
//     slab feeds the matrix cores; one barrier per slab;
//   * the product is formed transposed inside the MFMA (B fragment as the
//     first operand) so that a wave's result lanes run down a column: the
//     epilogue's loads and stores are 256-byte column segments;
//   * workgroup -> tile order keeps the tiles of one row panel of op(A) on
//     one XCD (consecutive tiles share the A panel in that XCD's L2);
//   * optional triangular structure of op(A) / op(B) trims each tile's K range;
//     optional split-K writes partial tiles that a reduction kernel combines
//     with the epilogue (small, deep products: Gram matrices, projections).
#include "gemm.hpp"

namespace chfsi {

namespace {

template <int OPA, int OPB, int BM, int BN, int BK>
struct ZTile {
  static constexpr int NT = 256;
  static constexpr int PAD = 1;
  static constexpr int LDA_S = BM + PAD;
  static constexpr int LDB_S = BN + PAD;
  static constexpr int EA = BM * BK / NT;  // A elements per thread per slab
  static constexpr int EB = BK * BN / NT;  // B elements per thread per slab
  static constexpr int MI = BM / 32;       // 16-row fragments per wave
  static constexpr int NJ = BN / 32;       // 16-col fragments per wave
  static_assert(EA >= 1 && EB >= 1, "tile too small for 256 threads");
  static_assert(BM * BK % NT == 0 && BK * BN % NT == 0, "tile/thread mismatch");
  static_assert(BK % 4 == 0, "BK multiple of the MFMA depth");
};

__device__ inline zc ld_z(const zc* p) { return *p; }

template <int OPA, int OPB, int BM, int BN, int BK>
__device__ __forceinline__ void zgemm_body(const ZGemmParams& p) {
  using T = ZTile<OPA, OPB, BM, BN, BK>;
  __shared__ zc As[2][BK][T::LDA_S];
  __shared__ zc Bs[2][BK][T::LDB_S];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int wm0 = (wave & 1) * (BM / 2);
  const int wn0 = (wave >> 1) * (BN / 2);

  // tile index with XCD-aware remap (workgroup i runs on XCD i % 8)
  const int64_t T_ = (int64_t)p.tiles_m * p.tiles_n;
  int64_t bid = blockIdx.x, t;
  const int64_t full = (T_ / 8) * 8;
  if (bid < full) t = (bid % 8) * (T_ / 8) + bid / 8;
  else t = bid;
  const int64_t mt = t / p.tiles_n, nt = t % p.tiles_n;
  const int64_t m0 = mt * BM, n0 = nt * BN;
  if ((p.flags & GEMM_OUT_LOWER) && n0 > m0 + BM - 1) return;  // tile entirely above the diagonal

  const int bz = blockIdx.y;
  const int batch = bz / p.splitk, split = bz % p.splitk;
  const zc* __restrict__ A = p.A + (int64_t)batch * p.sA;
  const zc* __restrict__ B = p.B + (int64_t)batch * p.sB;

  int64_t kbeg = 0, kend = p.K;
  if (p.flags & GEMM_TRI_A_LOWER) kend = min(kend, m0 + BM);
  if (p.flags & GEMM_TRI_A_UPPER) kbeg = max(kbeg, m0);
  if (p.flags & GEMM_TRI_B_UPPER) kend = min(kend, n0 + BN);
  if (p.flags & GEMM_TRI_B_LOWER) kbeg = max(kbeg, n0);
  if (p.splitk > 1) {
    kbeg = max(kbeg, (int64_t)split * p.kchunk);
    kend = min(kend, (int64_t)(split + 1) * p.kchunk);
  }
  const int64_t nslab = kend > kbeg ? cdiv(kend - kbeg, (int64_t)BK) : 0;

  d4v accR[T::MI][T::NJ], accI[T::MI][T::NJ];
#pragma unroll
  for (int i = 0; i < T::MI; i++)
#pragma unroll
    for (int j = 0; j < T::NJ; j++) {
      accR[i][j] = d4v{0.0, 0.0, 0.0, 0.0};
      accI[i][j] = d4v{0.0, 0.0, 0.0, 0.0};
    }

  zc ra[T::EA], rb[T::EB];

  auto load_slab = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < T::EA; q++) {
      const int e = tid + q * T::NT;
      int mm, kk;
      if (OPA == OP_N) { mm = e % BM; kk = e / BM; }
      else { kk = e % BK; mm = e / BK; }
      const int64_t gm = m0 + mm, gk = k0 + kk;
      zc v = zmk(0.0, 0.0);
      if (gm < p.M && gk < kend) {
        if (OPA == OP_N) v = A[gm + gk * p.lda];
        else v = zconj(A[gk + gm * p.lda]);
      }
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < T::EB; q++) {
      const int e = tid + q * T::NT;
      int kk, nn;
      if (OPB == OP_N) { kk = e % BK; nn = e / BK; }
      else { nn = e % BN; kk = e / BN; }
      const int64_t gn = n0 + nn, gk = k0 + kk;
      zc v = zmk(0.0, 0.0);
      if (gn < p.N && gk < kend) {
        if (OPB == OP_N) v = B[gk + gn * p.ldb];
        else v = zconj(B[gn + gk * p.ldb]);
      }
      rb[q] = v;
    }
  };
  auto store_slab = [&](int buf) {
#pragma unroll
    for (int q = 0; q < T::EA; q++) {
      const int e = tid + q * T::NT;
      int mm, kk;
      if (OPA == OP_N) { mm = e % BM; kk = e / BM; }
      else { kk = e % BK; mm = e / BK; }
      As[buf][kk][mm] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < T::EB; q++) {
      const int e = tid + q * T::NT;
      int kk, nn;
      if (OPB == OP_N) { kk = e % BK; nn = e / BK; }
      else { nn = e % BN; kk = e / BN; }
      Bs[buf][kk][nn] = rb[q];
    }
  };

  if (nslab > 0) {
    load_slab(kbeg);
    store_slab(0);
    __syncthreads();
    for (int64_t s = 0; s < nslab; s++) {
      const int buf = (int)(s & 1);
      if (s + 1 < nslab) load_slab(kbeg + (s + 1) * BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        zc a[T::MI], b[T::NJ];
#pragma unroll
        for (int i = 0; i < T::MI; i++) a[i] = As[buf][kk + lk][wm0 + i * 16 + lr];
#pragma unroll
        for (int j = 0; j < T::NJ; j++) b[j] = Bs[buf][kk + lk][wn0 + j * 16 + lr];
#pragma unroll
        for (int i = 0; i < T::MI; i++)
#pragma unroll
          for (int j = 0; j < T::NJ; j++) {
            // D[n][m] += B[k][n] A[m][k]  (transposed product: result lanes run down columns)
            accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[j].x, a[i].x, accR[i][j], 0, 0, 0);
            accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[j].y, a[i].x, accI[i][j], 0, 0, 0);
            accR[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-b[j].y, a[i].y, accR[i][j], 0, 0, 0);
            accI[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[j].x, a[i].y, accI[i][j], 0, 0, 0);
          }
      }
      if (s + 1 < nslab) store_slab(buf ^ 1);
      __syncthreads();
    }
  }

  // Epilogue.  Result lane layout of v_mfma_f64_16x16x4f64: lane l, value r
  // holds D[l/16 + 4r][l%16]; here D's row is the output column n and its
  // column the output row m.
  if (p.splitk > 1) {
    zc* P = p.P + ((int64_t)batch * p.splitk + split) * p.M * p.N;
#pragma unroll
    for (int i = 0; i < T::MI; i++)
#pragma unroll
      for (int j = 0; j < T::NJ; j++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int64_t m = m0 + wm0 + i * 16 + lr;
          const int64_t n = n0 + wn0 + j * 16 + lk + 4 * r;
          if (m < p.M && n < p.N) P[m + n * p.M] = zmk(accR[i][j][r], accI[i][j][r]);
        }
    return;
  }
  zc* C = p.C + (int64_t)batch * p.sC;
  const zc* X = p.X ? p.X + (int64_t)batch * p.sX : nullptr;
  const zc* Z = p.Z ? p.Z + (int64_t)batch * p.sZ : nullptr;
#pragma unroll
  for (int i = 0; i < T::MI; i++)
#pragma unroll
    for (int j = 0; j < T::NJ; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int64_t m = m0 + wm0 + i * 16 + lr;
        const int64_t n = n0 + wn0 + j * 16 + lk + 4 * r;
        if (m < p.M && n < p.N) {
          zc v = zmk(p.alpha * accR[i][j][r], p.alpha * accI[i][j][r]);
          if (X) v = zadd(v, zscale(p.beta, X[m + n * p.ldx]));
          if (Z) v = zadd(v, zscale(p.gamma, Z[m + n * p.ldz]));
          C[m + n * p.ldc] = v;
        }
      }
}

template <int OPA, int OPB, int BM, int BN, int BK>
__global__ void __launch_bounds__(256, 2) zgemm_kernel(ZGemmParams p) {
  zgemm_body<OPA, OPB, BM, BN, BK>(p);
}

// One degree step of the Chebyshev filter: the same body, launched under its
// own symbol so that profiles separate the filter from the other products.
template <int BM, int BN, int BK>
__global__ void __launch_bounds__(256, 2) chebyshev_step_f64(ZGemmParams p) {
  zgemm_body<OP_N, OP_N, BM, BN, BK>(p);
}

// Combine split-K partial tiles and apply the epilogue.
__global__ void zgemm_splitk_reduce(ZGemmParams p) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int batch = blockIdx.y;
  if (e >= p.M * p.N) return;
  const int64_t m = e % p.M, n = e / p.M;
  const zc* P = p.P + (int64_t)batch * p.splitk * p.M * p.N;
  double re = 0.0, im = 0.0;
  for (int s = 0; s < p.splitk; s++) {
    const zc v = P[(int64_t)s * p.M * p.N + e];
    re += v.x;
    im += v.y;
  }
  zc v = zmk(p.alpha * re, p.alpha * im);
  if (p.X) v = zadd(v, zscale(p.beta, p.X[(int64_t)batch * p.sX + m + n * p.ldx]));
  if (p.Z) v = zadd(v, zscale(p.gamma, p.Z[(int64_t)batch * p.sZ + m + n * p.ldz]));
  p.C[(int64_t)batch * p.sC + m + n * p.ldc] = v;
}

template <int OPA, int OPB, int BM, int BN, int BK>
void launch_cfg(ZGemmParams& p, int batch, bool filter_step, hipStream_t st) {
  p.tiles_m = (int)cdiv(p.M, BM);
  p.tiles_n = (int)cdiv(p.N, BN);
  dim3 grid((unsigned)((int64_t)p.tiles_m * p.tiles_n), (unsigned)(batch * p.splitk));
  if (OPA == OP_N && OPB == OP_N && filter_step)
    hipLaunchKernelGGL((chebyshev_step_f64<BM, BN, BK>), grid, dim3(256), 0, st, p);
  else
    hipLaunchKernelGGL((zgemm_kernel<OPA, OPB, BM, BN, BK>), grid, dim3(256), 0, st, p);
  CHFSI_CHECK_LAUNCH();
}

template <int BM, int BN, int BK>
void launch_ops(int opA, int opB, ZGemmParams& p, int batch, bool filter_step, hipStream_t st) {
  if (opA == OP_N && opB == OP_N) launch_cfg<OP_N, OP_N, BM, BN, BK>(p, batch, filter_step, st);
  else if (opA == OP_N && opB == OP_C) launch_cfg<OP_N, OP_C, BM, BN, BK>(p, batch, filter_step, st);
  else if (opA == OP_C && opB == OP_N) launch_cfg<OP_C, OP_N, BM, BN, BK>(p, batch, filter_step, st);
  else launch_cfg<OP_C, OP_C, BM, BN, BK>(p, batch, filter_step, st);
}

}  // namespace

void zgemm(const GemmOp& g, const GemmWork& w, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return;
  ZGemmParams p{};
  p.M = g.M; p.N = g.N; p.K = g.K;
  p.A = g.A; p.lda = g.lda; p.sA = g.sA;
  p.B = g.B; p.ldb = g.ldb; p.sB = g.sB;
  p.C = g.C; p.ldc = g.ldc; p.sC = g.sC;
  p.X = g.X; p.ldx = g.ldx; p.sX = g.sX;
  p.Z = g.Z; p.ldz = g.ldz; p.sZ = g.sZ;
  p.alpha = g.alpha; p.beta = g.beta; p.gamma = g.gamma;
  p.flags = g.flags;
  p.splitk = 1;
  p.kchunk = g.K;
  p.P = nullptr;
  const int batch = g.batch > 0 ? g.batch : 1;

  // tile shape: 64x64 when there are enough tiles to fill the chip
  const bool big = cdiv(g.M, 64) * cdiv(g.N, 64) * batch >= 192;
  const int bm = big ? 64 : 32, bn = big ? 64 : 32, bk = 16;
  int64_t tiles = cdiv(g.M, bm) * cdiv(g.N, bn) * batch;

  // split K for small, deep products (tiles < 1 per CU)
  if (g.allow_splitk && !(g.flags & GEMM_OUT_LOWER) && tiles < 256 && g.K >= 8 * bk && w.P) {
    int64_t want = cdiv(512, tiles);
    int64_t maxsplit = g.K / (4 * bk);  // at least 4 slabs per split
    int64_t cap = (int64_t)(w.P_elems / ((size_t)g.M * (size_t)g.N * (size_t)batch));
    int64_t sk = std::min(std::min(want, maxsplit), std::min(cap, (int64_t)64));
    if (sk >= 2) {
      p.splitk = (int)sk;
      p.kchunk = cdiv(cdiv(g.K, sk), bk) * bk;
      p.splitk = (int)cdiv(g.K, p.kchunk);
      p.P = w.P;
    }
  }
  if (big) launch_ops<64, 64, 16>(g.opA, g.opB, p, batch, g.filter_step, st);
  else launch_ops<32, 32, 16>(g.opA, g.opB, p, batch, g.filter_step, st);
  if (p.splitk > 1) {
    dim3 grid((unsigned)cdiv(g.M * g.N, 256), (unsigned)batch);
    hipLaunchKernelGGL(zgemm_splitk_reduce, grid, dim3(256), 0, st, p);
    CHFSI_CHECK_LAUNCH();
  }
}

}  // namespace chfsi
