// Complex FP64 GEMM on gfx950 matrix cores with a fused three-term epilogue.
//
//   out = alpha * op(A) op(B) + beta * X + gamma * Z      (alpha, beta, gamma real)
//
// This is the Chebyshev filter step of Algorithm 1 (eq. (2), scaled and
// shifted): with op = N, X = Y_i and Z = Y_{i-1}, one launch computes
// Y_{i+1} = alpha A Y_i + beta Y_i + gamma Y_{i-1} and writes it over Y_{i-1},
// so every degree step reads A, Y_i, Y_{i-1} and writes Y_{i+1} once.  The
// same kernel (other op / flag combinations) serves every other dense product
// of the solver (Cholesky updates, triangular inverse, reduction to standard
// form, Householder block updates, Rayleigh-Ritz, back-transform).
//
// Design (CDNA4):
//   * 256 threads = 4 waves in a 2x2 arrangement (4x1 for tiles 48 columns
//     wide); a workgroup owns a BM x BN complex output tile, each wave
//     (BM/2) x (BN/2) (or (BM/4) x BN) of it as 16x16 blocks;
//   * complex products as real v_mfma_f64_16x16x4f64 per 16x16x4 block:
//     four of them into separate real / imaginary accumulators, or, where
//     the registers allow, three (Gauss's 3M form: the sums of operand parts are
//     formed in registers and three accumulator sets combined at the end),
//     which removes a quarter of the matrix-core work; the rounding error
//     stays within a small constant of the four-product form's normwise
//     bound (Higham, "Stability of a method for multiplying complex
//     matrices with three real matrix multiplications", SIMAX 1992);
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
//     with the epilogue (small, deep products: Gram matrices, projections);
//   * FP32 steps may add a column-scaled fourth term rs[j] R(:, j): the
//     forcing of the recurrence the FP32 filter runs on the Ritz residual.
#include "gemm.hpp"

namespace chfsi {

namespace {

// Precision traits: element type, real type, accumulator and the matrix-core
// instruction.  Result lane layouts of the 16x16x4 instructions (lane l,
// value r): FP64 holds D[l/16 + 4r][l%16], FP32 holds D[4(l/16) + r][l%16].
struct PF64 {
  using E = zc;
  using R = double;
  using Acc = d4v;
  static __device__ __forceinline__ Acc mfma(R a, R b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int lk, int r) { return lk + 4 * r; }
  static __device__ __forceinline__ E mk(R x, R y) { return make_double2(x, y); }
};
struct PF32 {
  using E = cc;
  using R = float;
  using Acc = f4v;
  static __device__ __forceinline__ Acc mfma(R a, R b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int lk, int r) { return 4 * lk + r; }
  static __device__ __forceinline__ E mk(R x, R y) { return make_float2(x, y); }
};

template <int BM, int BN, int BK, int NW = 4>
struct ZTile {
  static constexpr int NT = 64 * NW;  // threads: NW waves
  static constexpr int PAD = 1;
  static constexpr int LDA_S = BM + PAD;
  static constexpr int LDB_S = BN + PAD;
  static constexpr int EA = BM * BK / NT;  // A elements per thread per slab
  static constexpr int EB = BK * BN / NT;  // B elements per thread per slab
  // waves along M: with four waves 2 (2x2) where half the tile width is a
  // whole number of 16-column fragments, else 4 (4x1, e.g. 48 columns);
  // with eight waves 2 (2x4: 32 x 16 per wave for a 64 x 64 tile)
  static constexpr int WMW = NW == 8 ? 2 : ((BN % 32 == 0) ? 2 : 4);
  static constexpr int WN = NW / WMW;               // waves along N
  static constexpr int MI = BM / (16 * WMW);        // 16-row fragments per wave
  static constexpr int NJ = BN / (16 * WN);         // 16-col fragments per wave
  static constexpr int KS = BK / 4;        // MFMA depth steps per slab
  static_assert(NW == 4 || NW == 8, "four or eight waves");
  static_assert(EA >= 1 && EB >= 1, "tile too small for the thread count");
  static_assert(BM * BK % NT == 0 && BK * BN % NT == 0, "tile/thread mismatch");
  static_assert(BK % 4 == 0, "BK multiple of the MFMA depth");
  static_assert(MI >= 1 && NJ >= 1 && BM % (16 * WMW) == 0 && BN % (16 * WN) == 0, "wave fragments");
};

// Workgroup -> tile order with the XCD-aware remap (workgroup i runs on XCD
// i % 8): each XCD works through a contiguous range of tiles, so tiles that
// share a row panel of op(A) meet in the same L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t ntiles) {
  const int64_t full = (ntiles / 8) * 8;
  return bid < full ? (bid % 8) * (ntiles / 8) + bid / 8 : bid;
}

template <class PT, int OPA, int OPB, int BM, int BN, int BK, bool G3 = false, int NW = 4>
__device__ __forceinline__ void zgemm_body(const ZGemmParams& p, int64_t t, int batch, int split) {
  using T = ZTile<BM, BN, BK, NW>;
  using E = typename PT::E;
  using R = typename PT::R;
  using Acc = typename PT::Acc;
  // B slabs are stored k-fastest (consecutive threads take consecutive k of
  // one column, which keeps the global loads in contiguous runs); the row
  // padding spreads the BK rows of a 16-lane (FP64) or 32-lane (FP32) store
  // group over distinct LDS banks
  constexpr int LDB = BN + (sizeof(E) == 16 ? (BK == 8 ? 2 : 1) : (BK == 8 ? 4 : 2));
  __shared__ E As[2][BK][T::LDA_S];
  __shared__ E Bs[2][BK][LDB];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int wm0 = (wave % T::WMW) * (BM / T::WMW);
  const int wn0 = (wave / T::WMW) * (BN / T::WN);

  const int64_t mt = t / p.tiles_n, nt = t % p.tiles_n;
  const int64_t m0 = mt * BM, n0 = nt * BN;
  if ((p.flags & GEMM_OUT_LOWER) && n0 > m0 + BM - 1) return;  // tile entirely above the diagonal

  const E* __restrict__ A = static_cast<const E*>(p.A) + (int64_t)batch * p.sA;
  const E* __restrict__ B = static_cast<const E*>(p.B) + (int64_t)batch * p.sB;

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

  // Four real products per complex product: accR, accI hold the real and
  // imaginary parts.  Three (G3): with a = ar + i ai, b = br + i bi,
  //   t1 = br (ar + ai), t2 = ar (bi - br), t3 = ai (br + bi),
  //   re = t1 - t3, im = t1 + t2,
  // accumulated in accR (t1), accI (t2) and acc3 (t3) and combined once at
  // the end; the sums of operand parts are formed in registers per step.
  constexpr int MI3 = G3 ? T::MI : 1, NJ3 = G3 ? T::NJ : 1;
  Acc accR[T::MI][T::NJ], accI[T::MI][T::NJ], acc3[MI3][NJ3];
#pragma unroll
  for (int i = 0; i < T::MI; i++)
#pragma unroll
    for (int j = 0; j < T::NJ; j++) {
      accR[i][j] = Acc{0, 0, 0, 0};
      accI[i][j] = Acc{0, 0, 0, 0};
    }
#pragma unroll
  for (int i = 0; i < MI3; i++)
#pragma unroll
    for (int j = 0; j < NJ3; j++) acc3[i][j] = Acc{0, 0, 0, 0};

  E ra[T::EA], rb[T::EB];

  auto load_slab = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < T::EA; q++) {
      const int e = tid + q * T::NT;
      int mm, kk;
      if (OPA == OP_N) { mm = e % BM; kk = e / BM; }
      else { kk = e % BK; mm = e / BK; }
      const int64_t gm = m0 + mm, gk = k0 + kk;
      E v = PT::mk(0, 0);
      if (gm < p.M && gk < kend) {
        if (OPA == OP_N) v = A[gm + gk * p.lda];
        else {
          v = A[gk + gm * p.lda];
          v.y = -v.y;
        }
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
      E v = PT::mk(0, 0);
      if (gn < p.N && gk < kend) {
        if (OPB == OP_N) v = B[gk + gn * p.ldb];
        else {
          v = B[gn + gk * p.ldb];
          v.y = -v.y;
        }
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

  // eight-wave FP64 tiles issue the global loads of slab s + 2 right after
  // storing slab s + 1 (early in slab s, see below) instead of at the start
  // of slab s + 1: the loads get more than a slab to arrive (0.5-0.8 % at
  // widths 256-660, none at narrower four-wave tiles)
  constexpr bool EARLY = sizeof(E) == 16 && T::KS > 1 && NW == 8;
  if (nslab > 0) {
    load_slab(kbeg);
    store_slab(0);
    __syncthreads();
    if (EARLY && nslab > 1) load_slab(kbeg + BK);
    for (int64_t s = 0; s < nslab; s++) {
      const int buf = (int)(s & 1);
      if (!EARLY && s + 1 < nslab) load_slab(kbeg + (s + 1) * BK);
      // fragments of depth step 0; the next step's are read while the
      // current step's products run
      E a[2][T::MI], b[2][T::NJ];
#pragma unroll
      for (int i = 0; i < T::MI; i++) a[0][i] = As[buf][lk][wm0 + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < T::NJ; j++) b[0][j] = Bs[buf][lk][wn0 + j * 16 + lr];
#pragma unroll
      for (int ks = 0; ks < T::KS; ks++) {
        // with three accumulator sets and four waves the registers for a
        // second set of fragments are not there: read each step's fragments
        // when it starts (the other resident waves cover the LDS latency);
        // eight waves hold a quarter of the tile each and keep both sets
        constexpr bool ONE_SET = G3 && NW == 4;
        const int c = ONE_SET ? 0 : (ks & 1);
        if (ONE_SET) {
          if (ks > 0) {
#pragma unroll
            for (int i = 0; i < T::MI; i++) a[0][i] = As[buf][ks * 4 + lk][wm0 + i * 16 + lr];
#pragma unroll
            for (int j = 0; j < T::NJ; j++) b[0][j] = Bs[buf][ks * 4 + lk][wn0 + j * 16 + lr];
          }
        } else if (ks + 1 < T::KS) {
#pragma unroll
          for (int i = 0; i < T::MI; i++) a[c ^ 1][i] = As[buf][(ks + 1) * 4 + lk][wm0 + i * 16 + lr];
#pragma unroll
          for (int j = 0; j < T::NJ; j++) b[c ^ 1][j] = Bs[buf][(ks + 1) * 4 + lk][wn0 + j * 16 + lr];
        }
        // D[n][m] += B[k][n] A[m][k]  (transposed product: result lanes run
        // down columns).  The real products are issued type by type so that
        // dependent accumulations are MI*NJ instructions apart.
        if constexpr (G3) {
          R sa[T::MI], db[T::NJ], sb[T::NJ];
#pragma unroll
          for (int i = 0; i < T::MI; i++) sa[i] = a[c][i].x + a[c][i].y;
#pragma unroll
          for (int j = 0; j < T::NJ; j++) {
            db[j] = b[c][j].y - b[c][j].x;
            sb[j] = b[c][j].x + b[c][j].y;
          }
#pragma unroll
          for (int i = 0; i < T::MI; i++)
#pragma unroll
            for (int j = 0; j < T::NJ; j++)
              accR[i][j] = PT::mfma(b[c][j].x, sa[i], accR[i][j]);
#pragma unroll
          for (int i = 0; i < T::MI; i++)
#pragma unroll
            for (int j = 0; j < T::NJ; j++)
              accI[i][j] = PT::mfma(db[j], a[c][i].x, accI[i][j]);
#pragma unroll
          for (int i = 0; i < MI3; i++)
#pragma unroll
            for (int j = 0; j < NJ3; j++)
              acc3[i][j] = PT::mfma(sb[j], a[c][i].y, acc3[i][j]);
        } else {
#pragma unroll
          for (int i = 0; i < T::MI; i++)
#pragma unroll
            for (int j = 0; j < T::NJ; j++)
              accR[i][j] = PT::mfma(b[c][j].x, a[c][i].x, accR[i][j]);
#pragma unroll
          for (int i = 0; i < T::MI; i++)
#pragma unroll
            for (int j = 0; j < T::NJ; j++)
              accI[i][j] = PT::mfma(b[c][j].y, a[c][i].x, accI[i][j]);
#pragma unroll
          for (int i = 0; i < T::MI; i++)
#pragma unroll
            for (int j = 0; j < T::NJ; j++)
              accR[i][j] = PT::mfma(-b[c][j].y, a[c][i].y, accR[i][j]);
#pragma unroll
          for (int i = 0; i < T::MI; i++)
#pragma unroll
            for (int j = 0; j < T::NJ; j++)
              accI[i][j] = PT::mfma(b[c][j].x, a[c][i].y, accI[i][j]);
        }
        // the next slab into the other LDS buffer (its last reads were in
        // the previous slab, before the last barrier): FP64 after the second
        // depth step, so that its stores are done before the barrier instead
        // of leading up to it (1-1.5 % per step), the eight-wave tile, whose
        // loads were issued a slab earlier, after the first (another
        // 0.7 %); FP32 after the last step (earlier was 2-4 % slower there)
        constexpr int STORE_AT = sizeof(E) == 16 && T::KS > 1 ? (NW == 8 ? 0 : 1) : T::KS - 1;
        if (ks == STORE_AT && s + 1 < nslab) store_slab(buf ^ 1);
        if (EARLY && ks == STORE_AT && s + 2 < nslab) load_slab(kbeg + (s + 2) * BK);
      }
      __syncthreads();
    }
  }

  if constexpr (G3) {
#pragma unroll
    for (int i = 0; i < MI3; i++)
#pragma unroll
      for (int j = 0; j < NJ3; j++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const R t1 = accR[i][j][r];
          accR[i][j][r] = t1 - acc3[i][j][r];
          accI[i][j][r] = t1 + accI[i][j][r];
        }
  }

  // Epilogue.  D's row is the output column n, its column the output row m.
  if (p.splitk > 1) {
    E* P = static_cast<E*>(p.P) + ((int64_t)batch * p.splitk + split) * p.M * p.N;
#pragma unroll
    for (int i = 0; i < T::MI; i++)
#pragma unroll
      for (int j = 0; j < T::NJ; j++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int64_t m = m0 + wm0 + i * 16 + lr;
          const int64_t n = n0 + wn0 + j * 16 + PT::out_row(lk, r);
          if (m < p.M && n < p.N) P[m + n * p.M] = PT::mk(accR[i][j][r], accI[i][j][r]);
        }
    return;
  }
  E* C = static_cast<E*>(p.C) + (int64_t)batch * p.sC;
  const E* X = p.X ? static_cast<const E*>(p.X) + (int64_t)batch * p.sX : nullptr;
  const E* Z = p.Z ? static_cast<const E*>(p.Z) + (int64_t)batch * p.sZ : nullptr;
  const R al = (R)p.alpha, be = (R)p.beta, ga = (R)p.gamma;
#pragma unroll
  for (int i = 0; i < T::MI; i++)
#pragma unroll
    for (int j = 0; j < T::NJ; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int64_t m = m0 + wm0 + i * 16 + lr;
        const int64_t n = n0 + wn0 + j * 16 + PT::out_row(lk, r);
        if (m < p.M && n < p.N) {
          R vx = al * accR[i][j][r], vy = al * accI[i][j][r];
          if (X) {
            const E x = X[m + n * p.ldx];
            vx += be * x.x;
            vy += be * x.y;
          }
          if (Z) {
            const E z = Z[m + n * p.ldz];
            vx += ga * z.x;
            vy += ga * z.y;
          }
          if constexpr (sizeof(E) == 8) {
            if (p.R) {
              const E rv = static_cast<const E*>(p.R)[m + n * p.ldr];
              const R sc = (R)p.rs[n];
              vx += sc * rv.x;
              vy += sc * rv.y;
            }
          }
          C[m + n * p.ldc] = PT::mk(vx, vy);
        }
      }
}

// Whether a tile configuration forms its complex products with three real
// products: wherever the third accumulator set fits the registers the
// configuration's occupancy leaves (FP64: tiles up to 64 x 80 at two
// workgroups per CU; FP32 accumulators take half the registers).
template <class PT, int BM, int BN, int MINB>
constexpr bool gauss3() {
  return sizeof(typename PT::E) == 8 || (BM * BN <= 64 * 80 && MINB <= 2);
}

#define ZGEMM_TILE_ARGS(p) xcd_tile(blockIdx.x, (int64_t)(p).tiles_m * (p).tiles_n), \
                                 (int)(blockIdx.y / (p).splitk), (int)(blockIdx.y % (p).splitk)

// Products whose tile rows carry unequal work: a triangular op(A) gives
// row panel i a K range proportional to i + 1 (lower) or to the rows below
// it (upper), and a product restricted to the lower output tiles gives the
// bottom rows the most tiles (with an upper-triangular op(B), also the
// longest).  Their rows are
// taken in the order heaviest, lightest, second heaviest, second lightest,
// ..., so that each XCD's contiguous range of the order holds balanced work
// (in row order the XCD holding the heavy rows would finish last, alone);
// inside an XCD the workgroups resident on one CU are spread over the range
// (consecutive workgroups of an XCD go to different CUs), so a row-major
// walk gives every CU a share of heavy and light rows.
__device__ __forceinline__ int64_t balanced_rows(const ZGemmParams& p, int64_t t) {
  const bool lower_heavy = (p.flags & (GEMM_TRI_A_LOWER | GEMM_OUT_LOWER)) != 0;
  const bool upper_heavy = (p.flags & GEMM_TRI_A_UPPER) != 0;
  if (!lower_heavy && !upper_heavy) return t;
  const int64_t i = t / p.tiles_n, c = t - i * p.tiles_n;
  const int64_t heavy = lower_heavy ? p.tiles_m - 1 - (i >> 1) : (i >> 1);
  const int64_t light = lower_heavy ? (i >> 1) : p.tiles_m - 1 - (i >> 1);
  return ((i & 1) ? light : heavy) * p.tiles_n + c;
}

template <int OPA, int OPB, int BM, int BN, int BK, int MINB, int NW = 4>
__global__ void __launch_bounds__(64 * NW, MINB) zgemm_kernel(ZGemmParams p) {
  const int64_t t = balanced_rows(p, xcd_tile(blockIdx.x, (int64_t)p.tiles_m * p.tiles_n));
  zgemm_body<PF64, OPA, OPB, BM, BN, BK, gauss3<PF64, BM, BN, MINB>(), NW>(p, t, (int)(blockIdx.y / p.splitk),
                                                                           (int)(blockIdx.y % p.splitk));
}

// One degree step of the Chebyshev filter: the same body, launched under its
// own symbol so that profiles separate the filter from the other products.
template <int BM, int BN, int BK, int MINB, int NW = 4>
__global__ void __launch_bounds__(64 * NW, MINB) chebyshev_step_f64(ZGemmParams p) {
  zgemm_body<PF64, OP_N, OP_N, BM, BN, BK, gauss3<PF64, BM, BN, MINB>(), NW>(p, ZGEMM_TILE_ARGS(p));
}

// The mixed-precision filter step: complex FP32 operands on the FP32 matrix
// cores with FP32 accumulation.
template <int BM, int BN, int BK, int MINB, int NW = 4>
__global__ void __launch_bounds__(64 * NW, MINB) chebyshev_step_f32(ZGemmParams p) {
  zgemm_body<PF32, OP_N, OP_N, BM, BN, BK, gauss3<PF32, BM, BN, MINB>(), NW>(p, ZGEMM_TILE_ARGS(p));
}

// One degree step for a batch of problems of different sizes in one
// persistent launch: gp[g] describes problem g's step (no split), tile0[g]
// its first tile in the batch-wide tile range (tile0[G] = total; a problem
// with no work this step has tile0[g] == tile0[g + 1]).  The tile range is
// cut into blocks of GROUP_TILES consecutive tiles (tiles of one row panel
// of A are consecutive) dealt round-robin to the 8 XCDs, so every XCD gets
// a share of every problem (problems differ in K, so contiguous shares
// would leave XCDs idle); within its XCD (workgroup i runs on XCD i % 8) a
// workgroup takes the next tile of that XCD's sequence from a counter, so
// workgroups that drew cheap tiles take more.  ctr (8 ints per launch) must
// be zero at launch.  The grid is a fixed multiple of 8, so the launch does
// not depend on the problems' sizes and a captured graph of these launches
// stays valid while the active widths shrink.
constexpr int GROUP_TILES = 16;

template <class PT, int BM, int BN, int BK, int MINB, int NW>
__device__ __forceinline__ void grouped_body(const ZGemmParams* __restrict__ gp, const int64_t* __restrict__ tile0,
                                             int G, int* __restrict__ ctr) {
  __shared__ int64_t next;
  const int64_t total = tile0[G];
  const int xcd = blockIdx.x % 8;
  for (;;) {
    if (threadIdx.x == 0) {
      const int64_t i = atomicAdd(ctr + xcd, 1);
      next = ((i / GROUP_TILES) * 8 + xcd) * GROUP_TILES + i % GROUP_TILES;
    }
    __syncthreads();
    const int64_t t = next;
    __syncthreads();  // every thread has read `next` before it is rewritten
    if (t >= total) break;
    // last g with tile0[g] <= t (that problem has at least one tile)
    int lo = 0, hi = G - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tile0[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    // work item -> (row panel, K chunk, column tile): consecutive items share
    // the A sub-panel of one row panel and K chunk
    const ZGemmParams& p = gp[lo];
    const int64_t w = t - tile0[lo];
    const int64_t nt = w % p.tiles_n, rest = w / p.tiles_n;
    const int split = (int)(rest % p.splitk);
    const int64_t mt = rest / p.splitk;
    zgemm_body<PT, OP_N, OP_N, BM, BN, BK, gauss3<PT, BM, BN, MINB>(), NW>(p, mt * p.tiles_n + nt, 0, split);
    __syncthreads();  // LDS of this tile fully consumed before the next one
  }
}

template <int BM, int BN, int BK, int MINB, int NW = 4>
__global__ void __launch_bounds__(64 * NW, MINB) chebyshev_step_grouped_f64(const ZGemmParams* __restrict__ gp,
                                                                       const int64_t* __restrict__ tile0, int G,
                                                                       int* __restrict__ ctr) {
  grouped_body<PF64, BM, BN, BK, MINB, NW>(gp, tile0, G, ctr);
}

template <int BM, int BN, int BK, int MINB, int NW = 4>
__global__ void __launch_bounds__(64 * NW, MINB) chebyshev_step_grouped_f32(const ZGemmParams* __restrict__ gp,
                                                                       const int64_t* __restrict__ tile0, int G,
                                                                       int* __restrict__ ctr) {
  grouped_body<PF32, BM, BN, BK, MINB, NW>(gp, tile0, G, ctr);
}

// Combine split-K partial tiles and apply the epilogue (element e of batch
// entry `batch`).
template <class PT>
__device__ __forceinline__ void splitk_reduce_elem(const ZGemmParams& p, int64_t e, int batch) {
  using E = typename PT::E;
  using R = typename PT::R;
  const int64_t m = e % p.M, n = e / p.M;
  // lower-triangle products: the tiles above the diagonal wrote no partials
  if ((p.flags & GEMM_OUT_LOWER) && m < n) return;
  const E* P = static_cast<const E*>(p.P) + (int64_t)batch * p.splitk * p.M * p.N;
  R re = 0, im = 0;
  // unrolled so that several partial loads are in flight; the sum is still
  // taken in split order
#pragma unroll 8
  for (int s = 0; s < p.splitk; s++) {
    const E v = P[(int64_t)s * p.M * p.N + e];
    re += v.x;
    im += v.y;
  }
  R vx = (R)p.alpha * re, vy = (R)p.alpha * im;
  if (p.X) {
    const E x = static_cast<const E*>(p.X)[(int64_t)batch * p.sX + m + n * p.ldx];
    vx += (R)p.beta * x.x;
    vy += (R)p.beta * x.y;
  }
  if (p.Z) {
    const E z = static_cast<const E*>(p.Z)[(int64_t)batch * p.sZ + m + n * p.ldz];
    vx += (R)p.gamma * z.x;
    vy += (R)p.gamma * z.y;
  }
  if constexpr (sizeof(E) == 8) {
    if (p.R) {
      const E rv = static_cast<const E*>(p.R)[m + n * p.ldr];
      const R sc = (R)p.rs[n];
      vx += sc * rv.x;
      vy += sc * rv.y;
    }
  }
  static_cast<E*>(p.C)[(int64_t)batch * p.sC + m + n * p.ldc] = PT::mk(vx, vy);
}

template <class PT>
__device__ __forceinline__ void splitk_reduce_body(const ZGemmParams& p) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p.M * p.N) return;
  splitk_reduce_elem<PT>(p, e, blockIdx.y);
}

// The combination of a grouped step's split problems: elem0 is the
// (G + 1)-prefix of the elements M * N of the problems that were split
// (0 for the others); grid-stride over the total.
template <class PT>
__device__ __forceinline__ void grouped_reduce_body(const ZGemmParams* __restrict__ gp,
                                                    const int64_t* __restrict__ elem0, int G) {
  const int64_t total = elem0[G];
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = G - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (elem0[mid] <= e) lo = mid;
      else hi = mid - 1;
    }
    splitk_reduce_elem<PT>(gp[lo], e - elem0[lo], 0);
  }
}

__global__ void __launch_bounds__(256) chebyshev_step_grouped_reduce_f64(const ZGemmParams* __restrict__ gp,
                                                                         const int64_t* __restrict__ elem0, int G) {
  grouped_reduce_body<PF64>(gp, elem0, G);
}

__global__ void __launch_bounds__(256) chebyshev_step_grouped_reduce_f32(const ZGemmParams* __restrict__ gp,
                                                                         const int64_t* __restrict__ elem0, int G) {
  grouped_reduce_body<PF32>(gp, elem0, G);
}

__global__ void zgemm_splitk_reduce(ZGemmParams p) { splitk_reduce_body<PF64>(p); }

// The filter steps' split-K combinations (own symbols, like the steps).
__global__ void chebyshev_step_reduce_f64(ZGemmParams p) { splitk_reduce_body<PF64>(p); }
__global__ void chebyshev_step_reduce_f32(ZGemmParams p) { splitk_reduce_body<PF32>(p); }

// Tile configurations.  All use 256 threads (2x2 waves; 4x1 for 48 columns).
struct Cfg {
  int bm, bn, bk, minb;
  double eff;  // relative per-tile efficiency used by the chooser
};
constexpr Cfg CFGS[] = {
    {0, 0, 0, 0, 0.0},        // 0: automatic
    {64, 64, 16, 2, 1.0},     // 1
    {32, 32, 16, 2, 0.55},    // 2
    {64, 64, 8, 2, 1.0},      // 3
    {128, 64, 8, 2, 1.05},    // 4
    {64, 128, 8, 2, 1.05},    // 5
    {128, 128, 8, 1, 1.1},    // 6
    {64, 32, 16, 2, 0.8},     // 7
    {64, 64, 8, 4, 1.0},      // 8: as 3 with room for four workgroups per CU
    {64, 32, 16, 4, 0.8},     // 9: as 7 with room for four workgroups per CU
    {64, 48, 16, 2, 0.9},     // 10: 48 columns (4x1 waves) for active widths that pad 64 / 32
    {64, 64, 16, 2, 1.04},    // 11: as 1 with eight waves (2x4, 32 x 16 per wave)
    {64, 80, 16, 2, 1.0},     // 12: 80 columns (4x1 waves, 16 x 80 each)
};
constexpr int NCFG = sizeof(CFGS) / sizeof(CFGS[0]);

template <int OPA, int OPB, int BM, int BN, int BK, int MINB, int NW = 4>
void launch_one(ZGemmParams& p, int batch, bool filter_step, hipStream_t st) {
  p.tiles_m = (int)cdiv(p.M, BM);
  p.tiles_n = (int)cdiv(p.N, BN);
  dim3 grid((unsigned)((int64_t)p.tiles_m * p.tiles_n), (unsigned)(batch * p.splitk));
  if (OPA == OP_N && OPB == OP_N && filter_step)
    hipLaunchKernelGGL((chebyshev_step_f64<BM, BN, BK, MINB, NW>), grid, dim3(64 * NW), 0, st, p);
  else
    hipLaunchKernelGGL((zgemm_kernel<OPA, OPB, BM, BN, BK, MINB, NW>), grid, dim3(64 * NW), 0, st, p);
  CHFSI_CHECK_LAUNCH();
}

template <int BM, int BN, int BK, int MINB, int NW = 4>
void launch_one_f32(ZGemmParams& p, int batch, hipStream_t st) {
  p.tiles_m = (int)cdiv(p.M, BM);
  p.tiles_n = (int)cdiv(p.N, BN);
  dim3 grid((unsigned)((int64_t)p.tiles_m * p.tiles_n), (unsigned)(batch * p.splitk));
  hipLaunchKernelGGL((chebyshev_step_f32<BM, BN, BK, MINB, NW>), grid, dim3(64 * NW), 0, st, p);
  CHFSI_CHECK_LAUNCH();
}

void launch_f32(int cfg, ZGemmParams& p, int batch, hipStream_t st) {
  switch (cfg) {
    case 1: launch_one_f32<64, 64, 16, 2>(p, batch, st); break;
    case 2: launch_one_f32<32, 32, 16, 2>(p, batch, st); break;
    case 3: launch_one_f32<64, 64, 8, 2>(p, batch, st); break;
    case 4: launch_one_f32<128, 64, 8, 2>(p, batch, st); break;
    case 5: launch_one_f32<64, 128, 8, 2>(p, batch, st); break;
    case 6: launch_one_f32<128, 128, 8, 1>(p, batch, st); break;
    case 7: launch_one_f32<64, 32, 16, 2>(p, batch, st); break;
    case 8: launch_one_f32<64, 64, 8, 4>(p, batch, st); break;
    case 9: launch_one_f32<64, 32, 16, 4>(p, batch, st); break;
    case 10: launch_one_f32<64, 48, 16, 2>(p, batch, st); break;
    case 11: launch_one_f32<64, 64, 16, 2, 8>(p, batch, st); break;
    case 12: launch_one_f32<64, 80, 16, 2>(p, batch, st); break;
    default: throw Error(ST_EINVAL, "cgemm: bad tile configuration");
  }
}

template <int OPA, int OPB>
void launch_cfg(int cfg, ZGemmParams& p, int batch, bool filter_step, hipStream_t st) {
  switch (cfg) {
    case 1: launch_one<OPA, OPB, 64, 64, 16, 2>(p, batch, filter_step, st); break;
    case 2: launch_one<OPA, OPB, 32, 32, 16, 2>(p, batch, filter_step, st); break;
    case 7: launch_one<OPA, OPB, 64, 32, 16, 2>(p, batch, filter_step, st); break;
    case 11: launch_one<OPA, OPB, 64, 64, 16, 2, 8>(p, batch, filter_step, st); break;
    default:
      if constexpr (OPA == OP_N && OPB == OP_N) {
        switch (cfg) {
          case 3: launch_one<OPA, OPB, 64, 64, 8, 2>(p, batch, filter_step, st); return;
          case 4: launch_one<OPA, OPB, 128, 64, 8, 2>(p, batch, filter_step, st); return;
          case 5: launch_one<OPA, OPB, 64, 128, 8, 2>(p, batch, filter_step, st); return;
          case 6: launch_one<OPA, OPB, 128, 128, 8, 1>(p, batch, filter_step, st); return;
          case 8: launch_one<OPA, OPB, 64, 64, 8, 4>(p, batch, filter_step, st); return;
          case 9: launch_one<OPA, OPB, 64, 32, 16, 4>(p, batch, filter_step, st); return;
          case 10: launch_one<OPA, OPB, 64, 48, 16, 2>(p, batch, filter_step, st); return;
          case 12: launch_one<OPA, OPB, 64, 80, 16, 2>(p, batch, filter_step, st); return;
          default: break;
        }
      }
      throw Error(ST_EINVAL, "zgemm: tile configuration " + std::to_string(cfg) + " not available for these ops");
  }
}

void launch_ops(int cfg, int opA, int opB, ZGemmParams& p, int batch, bool filter_step, hipStream_t st) {
  if (opA == OP_N && opB == OP_N) launch_cfg<OP_N, OP_N>(cfg, p, batch, filter_step, st);
  else if (opA == OP_N && opB == OP_C) launch_cfg<OP_N, OP_C>(cfg, p, batch, filter_step, st);
  else if (opA == OP_C && opB == OP_N) launch_cfg<OP_C, OP_N>(cfg, p, batch, filter_step, st);
  else launch_cfg<OP_C, OP_C>(cfg, p, batch, filter_step, st);
}

template <int BM, int BN, int BK, int MINB, int NW = 4>
void launch_grouped(int prec, const ZGemmParams* gp, const int64_t* tile0, int G, int* ctr, int grid, hipStream_t st) {
  if (prec == PREC_F32)
    hipLaunchKernelGGL((chebyshev_step_grouped_f32<BM, BN, BK, MINB, NW>), dim3(grid), dim3(64 * NW), 0, st, gp, tile0,
                       G, ctr);
  else
    hipLaunchKernelGGL((chebyshev_step_grouped_f64<BM, BN, BK, MINB, NW>), dim3(grid), dim3(64 * NW), 0, st, gp, tile0,
                       G, ctr);
  CHFSI_CHECK_LAUNCH();
}

// Resident workgroups per CU of the grouped kernel.
template <int BM, int BN, int BK, int MINB, int NW = 4>
int grouped_occupancy(int prec) {
  int nb = 0;
  if (prec == PREC_F32)
    CHFSI_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, chebyshev_step_grouped_f32<BM, BN, BK, MINB, NW>,
                                                           64 * NW, 0));
  else
    CHFSI_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, chebyshev_step_grouped_f64<BM, BN, BK, MINB, NW>,
                                                           64 * NW, 0));
  return nb;
}

}  // namespace

int zgemm_num_configs() { return NCFG; }

int zgemm_tile_shape(int cfg, int* bm, int* bn) {
  if (cfg < 1 || cfg >= NCFG) return -1;
  *bm = CFGS[cfg].bm;
  *bn = CFGS[cfg].bn;
  return 0;
}

void zgemm_grouped_reduce(int prec, const ZGemmParams* gp, const int64_t* elem0, int G, int grid, hipStream_t st) {
  if (grid < 1 || G < 1) throw Error(ST_EINVAL, "grouped reduce: bad grid or no problems");
  if (prec == PREC_F32)
    hipLaunchKernelGGL(chebyshev_step_grouped_reduce_f32, dim3(grid), dim3(256), 0, st, gp, elem0, G);
  else
    hipLaunchKernelGGL(chebyshev_step_grouped_reduce_f64, dim3(grid), dim3(256), 0, st, gp, elem0, G);
  CHFSI_CHECK_LAUNCH();
}

int zgemm_config_bk(int cfg) { return (cfg >= 1 && cfg < NCFG) ? CFGS[cfg].bk : 0; }

bool zgemm_grouped_config_ok(int cfg) {
  return cfg == 1 || cfg == 2 || cfg == 3 || cfg == 4 || cfg == 5 || cfg == 7 || cfg == 11 || cfg == 12;
}

int zgemm_grouped_grid(int prec, int cfg) {
  int nb = 0;
  switch (cfg) {
    case 1: nb = grouped_occupancy<64, 64, 16, 2>(prec); break;
    case 2: nb = grouped_occupancy<32, 32, 16, 2>(prec); break;
    case 3: nb = grouped_occupancy<64, 64, 8, 2>(prec); break;
    case 4: nb = grouped_occupancy<128, 64, 8, 2>(prec); break;
    case 5: nb = grouped_occupancy<64, 128, 8, 2>(prec); break;
    case 7: nb = grouped_occupancy<64, 32, 16, 2>(prec); break;
    case 11: nb = grouped_occupancy<64, 64, 16, 2, 8>(prec); break;
    case 12: nb = grouped_occupancy<64, 80, 16, 2>(prec); break;
    default: throw Error(ST_EINVAL, "grouped filter: bad tile configuration");
  }
  int dev = 0, cus = 0;
  CHFSI_HIP(hipGetDevice(&dev));
  CHFSI_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int grid = std::max(1, nb) * std::max(1, cus);
  return std::max(8, grid / 8 * 8);
}

void zgemm_grouped_filter_step(int prec, int cfg, const ZGemmParams* gp, const int64_t* tile0, int G, int* ctr,
                               int grid, hipStream_t st) {
  if (grid < 8 || grid % 8) throw Error(ST_EINVAL, "grouped filter: grid must be a positive multiple of 8");
  if (G < 1 || !ctr) throw Error(ST_EINVAL, "grouped filter: no problems or no counters");
  switch (cfg) {
    case 1: launch_grouped<64, 64, 16, 2>(prec, gp, tile0, G, ctr, grid, st); break;
    case 2: launch_grouped<32, 32, 16, 2>(prec, gp, tile0, G, ctr, grid, st); break;
    case 3: launch_grouped<64, 64, 8, 2>(prec, gp, tile0, G, ctr, grid, st); break;
    case 4: launch_grouped<128, 64, 8, 2>(prec, gp, tile0, G, ctr, grid, st); break;
    case 5: launch_grouped<64, 128, 8, 2>(prec, gp, tile0, G, ctr, grid, st); break;
    case 7: launch_grouped<64, 32, 16, 2>(prec, gp, tile0, G, ctr, grid, st); break;
    case 11: launch_grouped<64, 64, 16, 2, 8>(prec, gp, tile0, G, ctr, grid, st); break;
    case 12: launch_grouped<64, 80, 16, 2>(prec, gp, tile0, G, ctr, grid, st); break;
    default: throw Error(ST_EINVAL, "grouped filter: bad tile configuration");
  }
}

// Choose the tile configuration and the K split: maximise the estimated
// throughput = per-tile efficiency x occupancy of the chip's workgroup slots
// (256 CUs x workgroups per CU), charging split-K for its partial-tile traffic.
// Cost per computed column of the 48- and 32-wide filter tiles relative to
// the 64-wide eight-wave tile's (FP64, tall deep products; sweeps of active
// widths 16 to 660 at n = 4000 and 10000 on MI355X, every tile with its
// best K split: the 64-wide tile with eight waves runs 3-5 % faster than
// with four, and the 48-wide tile's 4x1 waves read more LDS per matrix-core
// product).  With these weights the rule picks the fastest shape at every
// width of the sweeps but one (within 3 % there).
constexpr double W48_COST = 1.14, W32_COST = 1.12;
// The same for the FP32 tiles (a sweep of active widths 40 to 440 at
// n = 4000).
constexpr double W48_COST_F32 = 1.07, W32_COST_F32 = 1.08;
// The 80-wide tile (4x1 waves, 16 x 80 each), FP64 and FP32: from sweeps of
// widths 70 to 640 at n = 4000 and 10000 against every other width at its
// best K split (16-20 % faster at 65-80 columns, 4 % at 400).
constexpr double W80_COST = 1.06, W80_COST_F32 = 1.03;

void zgemm_choose(const GemmOp& g, int64_t P_elems, int& cfg, int& splitk) {
  const int batch = g.batch > 0 ? g.batch : 1;
  const bool nn = g.opA == OP_N && g.opB == OP_N;
  // Tall, deep products (the filter's A Y_i and the Rayleigh-Ritz A Q): rules
  // read off sweeps of the configurations and splits on MI355X (n = 2000,
  // 4000 and 10000, k_a from 16 to 660).  The 64 x 64 x 16 tile (FP64 with
  // eight waves) leads unless its last column tile pads N clearly more than
  // the narrower tiles do.  K is split so that each workgroup's range stays near 1000 (the A
  // panels of the workgroups resident on one XCD then fit its 4 MB L2), and
  // further where the tiles alone would leave the CUs short of work (FP32
  // steps are shorter and want about twice as many workgroups).  The tile
  // width (80, 64, 48 or 32 columns) that computes the fewest padded columns,
  // each width's columns weighted by its measured cost relative to the
  // 64-wide tile's (per precision).
  if (nn && batch == 1 && g.M >= 1024 && g.K >= 1024 && !(g.flags & GEMM_OUT_LOWER)) {
    const bool f32 = g.prec == PREC_F32;
    const double pad64 = (double)(cdiv(g.N, (int64_t)64) * 64) / (double)g.N;
    const double pad32 = (double)(cdiv(g.N, (int64_t)32) * 32) / (double)g.N;
    const double pad48 = (double)(cdiv(g.N, (int64_t)48) * 48) / (double)g.N;
    const double pad80 = (double)(cdiv(g.N, (int64_t)80) * 80) / (double)g.N;
    const double cost64 = pad64, cost48 = (f32 ? W48_COST_F32 : W48_COST) * pad48,
                 cost32 = (f32 ? W32_COST_F32 : W32_COST) * pad32, cost80 = (f32 ? W80_COST_F32 : W80_COST) * pad80;
    // (FP64: the 64-wide tile with eight waves; FP32 keeps four)
    int c = cost64 <= cost48 && cost64 <= cost32 ? (f32 ? 1 : 11) : (cost48 <= cost32 ? 10 : 7);
    if (cost80 < std::min(cost64, std::min(cost48, cost32))) c = 12;
    // (FP32 blocks of 97-128 columns: the 64 x 128 x 8 tile, one column tile)
    if (f32 && g.N > 96 && g.N <= 128) c = 5;
    int sk = g.K < 1500 ? 1 : g.K < 3000 ? 2 : g.K < 7000 ? 4 : 8;
    if (f32) sk = std::min(8, 2 * sk);
    const int64_t tiles = cdiv(g.M, (int64_t)CFGS[c].bm) * cdiv(g.N, (int64_t)CFGS[c].bn);
    const int64_t want = f32 ? 1000 : 480;
    while (sk < 8 && tiles * sk < want && g.K >= (int64_t)2 * sk * (f32 ? 200 : 250)) sk *= 2;
    // a triangular op(A) leaves the top row panels short: deeper splits
    // rebalance the workgroups
    if (g.flags & (GEMM_TRI_A_LOWER | GEMM_TRI_A_UPPER)) sk = std::min(16, 2 * sk);
    const size_t cap = (size_t)P_elems * (f32 ? 2 : 1);
    while (sk > 1 && (!g.allow_splitk || !P_elems || (size_t)sk * g.M * g.N > cap ||
                      g.K < (int64_t)sk * 4 * CFGS[c].bk))
      sk /= 2;
    cfg = c;
    splitk = sk;
    return;
  }
  // Small outputs of deep products (Gram matrices Y^H Y, Q^H W, full or
  // lower triangle): 32 x 32 tiles split 16 ways, and further (up to 64,
  // each split at least two slabs deep) while the tiles and splits give
  // fewer than 256 workgroups; tall products with a short K (n x k times
  // k x k): 32 x 32 tiles, no split (both read off the same sweep).
  const int gram_struct = g.flags & ~GEMM_OUT_LOWER;
  if (batch == 1 && g.M * g.N <= 512 * 512 && g.K >= 2048 && g.allow_splitk && P_elems && !gram_struct &&
      g.prec == PREC_F64) {
    const int64_t tm = cdiv(g.M, (int64_t)32), tn = cdiv(g.N, (int64_t)32);
    const int64_t tiles = (g.flags & GEMM_OUT_LOWER) && tm == tn ? tm * (tm + 1) / 2 : tm * tn;
    int sk = 16;
    while (sk < 64 && tiles * sk < 256 && g.K >= (int64_t)2 * sk * 2 * CFGS[2].bk) sk *= 2;
    const int min_slabs = sk > 16 ? 2 : 4;
    while (sk > 1 && ((size_t)sk * g.M * g.N > (size_t)P_elems || g.K < (int64_t)sk * min_slabs * CFGS[2].bk)) sk /= 2;
    cfg = 2;
    splitk = sk;
    return;
  }
  if (batch == 1 && g.K <= 512 && g.M >= 1024 && g.N <= 512) {
    cfg = 2;
    splitk = 1;
    return;
  }
  double best = -1.0;
  cfg = 1;
  splitk = 1;
  const int cands_nn[] = {1, 2, 4, 5, 7};
  const int cands_other[] = {1, 2, 7, 11};
  const int* cands = nn ? cands_nn : cands_other;
  const int ncand = nn ? 5 : 4;
  for (int ci = 0; ci < ncand; ci++) {
    const Cfg& c = CFGS[cands[ci]];
    const int64_t tiles = cdiv(g.M, c.bm) * cdiv(g.N, c.bn) * batch;
    const int64_t slots = 256LL * c.minb;
    // useful fraction of the tile (ragged edges)
    const double fill = (double)(g.M * g.N) / (double)(cdiv(g.M, c.bm) * c.bm * cdiv(g.N, c.bn) * c.bn);
    for (int sk = 1; sk <= 16; sk *= 2) {
      if (sk > 1) {
        if (!g.allow_splitk || (g.flags & GEMM_OUT_LOWER) || !P_elems) break;
        if (g.K < (int64_t)sk * 4 * c.bk) break;
        if ((size_t)sk * g.M * g.N * batch > (size_t)P_elems) break;
      }
      const int64_t work = tiles * sk;
      const double waves = std::ceil((double)work / (double)slots);
      const double occ = (double)work / (waves * (double)slots);
      // split-K traffic relative to the product's own reads
      const double extra = sk > 1 ? (double)sk * 2.0 * g.M * g.N / (double)(g.M * g.K + g.K * g.N + 1) : 0.0;
      const double score = c.eff * fill * occ / (1.0 + 0.5 * extra);
      if (score > best * 1.02) {
        best = score;
        cfg = cands[ci];
        splitk = sk;
      }
    }
  }
}

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
  const int batch = g.batch > 0 ? g.batch : 1;

  int cfg = g.cfg, sk = g.splitk;
  if (cfg < 0 || cfg >= NCFG || sk < 0) throw Error(ST_EINVAL, "zgemm: bad tile configuration or split");
  if (cfg == 0 || sk == 0) {
    int c2, s2;
    zgemm_choose(g, w.P ? (int64_t)w.P_elems : 0, c2, s2);
    if (cfg == 0) cfg = c2;
    if (sk == 0) sk = (g.cfg == 0) ? s2 : 1;
  }
  const bool f32 = g.prec == PREC_F32;
  if (f32 && (g.opA != OP_N || g.opB != OP_N || g.flags))
    throw Error(ST_EINVAL, "zgemm: FP32 products support op = N and no structure flags only");
  if (g.R && (!f32 || batch != 1 || !g.rs || g.ldr < g.M))
    throw Error(ST_EINVAL, "zgemm: the column-scaled term needs an FP32 product, batch 1, rs and ldr >= M");
  p.R = g.R; p.ldr = g.ldr; p.rs = g.rs;
  if (sk > 1) {
    const size_t cap = f32 ? 2 * w.P_elems : w.P_elems;
    if (!w.P || (size_t)sk * g.M * g.N * batch > cap)
      throw Error(ST_EINVAL, "zgemm: split-K scratch too small");
    const int bk = CFGS[cfg].bk;
    p.kchunk = cdiv(cdiv(g.K, sk), bk) * bk;
    p.splitk = (int)std::max<int64_t>(1, cdiv(g.K, p.kchunk));
    p.P = w.P;
  } else {
    p.splitk = 1;
    p.kchunk = g.K;
    p.P = nullptr;
  }
  if (f32) launch_f32(cfg, p, batch, st);
  else launch_ops(cfg, g.opA, g.opB, p, batch, g.filter_step, st);
  if (p.splitk > 1) {
    dim3 grid((unsigned)cdiv(g.M * g.N, 256), (unsigned)batch);
    if (f32) hipLaunchKernelGGL(chebyshev_step_reduce_f32, grid, dim3(256), 0, st, p);
    else if (g.filter_step) hipLaunchKernelGGL(chebyshev_step_reduce_f64, grid, dim3(256), 0, st, p);
    else hipLaunchKernelGGL(zgemm_splitk_reduce, grid, dim3(256), 0, st, p);
    CHFSI_CHECK_LAUNCH();
  }
}

}  // namespace chfsi
