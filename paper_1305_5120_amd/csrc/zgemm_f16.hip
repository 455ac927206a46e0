// Complex products with FP16 operands on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_f16: FP16 inputs, FP32 accumulation), for the degree
// steps of the filter's Ritz-residual recurrence in precision 3.
//
// With Y_0 Ritz vectors of A, the iterates of the recurrence of eq. (2)
// split as Y_i = Y_0 diag(t_i(mu)) + D_i; only the residual part D is formed
// with these products.  Its columns are scaled to unit size (by powers of
// two) before the first step, so FP16 holds their range, and its rounding
// errors stay relative to |D|, which shrinks with the residual: the
// filtered block keeps FP64 accuracy where Y_0 has converged.
//
// Operands: A in two FP16 planes (real parts, then imaginary parts), row m
// holding A(m, k) for consecutive k (a row-major copy, taken from the
// column-major Hermitian A by conjugation, with a zero-padded row length);
// D, the partial tiles and the output in complex FP32 (interleaved, column
// major).  One step computes
//   C = alpha A B + beta X + gamma Z + R diag(rs)
// over a 64 x 64 output tile per workgroup of four waves (2 x 2, 32 x 32
// each as 2 x 2 fragments of 16 x 16), K in slabs of 32 staged through LDS
// and double buffered; each complex product is four real products.  As in
// the FP64 and FP32 steps, the product is formed transposed inside the
// matrix instruction (the B fragment first), so a wave's result lanes run
// down an output column.
#include "gemm.hpp"

namespace chfsi {

namespace {

typedef _Float16 h8v __attribute__((ext_vector_type(8)));

constexpr int HB = 64;          // tile rows and columns
constexpr int HK = 32;          // slab depth (one matrix instruction per fragment pair and real product)
constexpr int HLD = HK + 8;     // LDS row stride in halves: 80 bytes, so 16 lanes' 16-byte reads hit distinct banks
constexpr int HNT = 256;        // threads

__device__ __forceinline__ int64_t xcd_tile_h(int64_t bid, int64_t ntiles) {
  const int64_t full = (ntiles / 8) * 8;
  return bid < full ? (bid % 8) * (ntiles / 8) + bid / 8 : bid;
}

__device__ __forceinline__ f4v mfma_h(h8v a, h8v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__global__ void __launch_bounds__(HNT, 2) chebyshev_step_f16(ZGemmParams p) {
  __shared__ __attribute__((aligned(16))) _Float16 As[2][2][HB][HLD];  // [buffer][re, im][row m][k]
  __shared__ __attribute__((aligned(16))) _Float16 Bs[2][2][HB][HLD];  // [buffer][re, im][column n][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int wm0 = (wave & 1) * 32, wn0 = (wave >> 1) * 32;

  const int64_t t = xcd_tile_h(blockIdx.x, (int64_t)p.tiles_m * p.tiles_n);
  const int64_t m0 = (t / p.tiles_n) * HB, n0 = (t % p.tiles_n) * HB;
  const int split = (int)blockIdx.y;
  const int64_t kbeg = (int64_t)split * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int64_t nslab = kend > kbeg ? cdiv(kend - kbeg, (int64_t)HK) : 0;

  const _Float16* __restrict__ Are = static_cast<const _Float16*>(p.A);
  const _Float16* __restrict__ Aim = Are + p.M * p.lda;
  const cc* __restrict__ B = static_cast<const cc*>(p.B);

  // this thread's share of a slab: row (A) / column (B) tid / 4, eight
  // consecutive k from 8 (tid % 4)
  const int lrow = tid >> 2, lk8 = (tid & 3) * 8;
  const int64_t gm = m0 + lrow, gn = n0 + lrow;
  uint4 ra_re, ra_im;
  h8v rb_re, rb_im;

  auto load_slab = [&](int64_t k0) {
    const int64_t k = k0 + lk8;
    // A: rows are zero-padded to lda (a multiple of 64) and chunk ends are
    // multiples of the slab depth, so only the row needs a check
    if (gm < p.M) {
      ra_re = *reinterpret_cast<const uint4*>(Are + gm * p.lda + k);
      ra_im = *reinterpret_cast<const uint4*>(Aim + gm * p.lda + k);
    } else {
      ra_re = make_uint4(0, 0, 0, 0);
      ra_im = make_uint4(0, 0, 0, 0);
    }
    if (gn < p.N && k + 8 <= kend) {
      const cc* col = B + gn * p.ldb + k;
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const cc v = col[j];
        rb_re[j] = (_Float16)v.x;
        rb_im[j] = (_Float16)v.y;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; j++) {
        cc v = make_float2(0.f, 0.f);
        if (gn < p.N && k + j < kend) v = B[gn * p.ldb + k + j];
        rb_re[j] = (_Float16)v.x;
        rb_im[j] = (_Float16)v.y;
      }
    }
  };
  auto store_slab = [&](int buf) {
    *reinterpret_cast<uint4*>(&As[buf][0][lrow][lk8]) = ra_re;
    *reinterpret_cast<uint4*>(&As[buf][1][lrow][lk8]) = ra_im;
    *reinterpret_cast<h8v*>(&Bs[buf][0][lrow][lk8]) = rb_re;
    *reinterpret_cast<h8v*>(&Bs[buf][1][lrow][lk8]) = rb_im;
  };

  f4v accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) {
      accR[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
      accI[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    }

  if (nslab > 0) {
    load_slab(kbeg);
    store_slab(0);
    __syncthreads();
    for (int64_t s = 0; s < nslab; s++) {
      const int buf = (int)(s & 1);
      if (s + 1 < nslab) load_slab(kbeg + (s + 1) * HK);
      h8v a_re[2], a_im[2], b_re[2], b_im[2], nb_im[2];
#pragma unroll
      for (int i = 0; i < 2; i++) {
        a_re[i] = *reinterpret_cast<const h8v*>(&As[buf][0][wm0 + 16 * i + lr][8 * lk]);
        a_im[i] = *reinterpret_cast<const h8v*>(&As[buf][1][wm0 + 16 * i + lr][8 * lk]);
      }
#pragma unroll
      for (int j = 0; j < 2; j++) {
        b_re[j] = *reinterpret_cast<const h8v*>(&Bs[buf][0][wn0 + 16 * j + lr][8 * lk]);
        b_im[j] = *reinterpret_cast<const h8v*>(&Bs[buf][1][wn0 + 16 * j + lr][8 * lk]);
        nb_im[j] = -b_im[j];
      }
      // D[n][m] += B[k][n] A[m][k]: re = Br Ar - Bi Ai, im = Bi Ar + Br Ai,
      // issued type by type (dependent accumulations four instructions apart)
#pragma unroll
      for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) accR[i][j] = mfma_h(b_re[j], a_re[i], accR[i][j]);
#pragma unroll
      for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) accI[i][j] = mfma_h(b_im[j], a_re[i], accI[i][j]);
#pragma unroll
      for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) accR[i][j] = mfma_h(nb_im[j], a_im[i], accR[i][j]);
#pragma unroll
      for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) accI[i][j] = mfma_h(b_re[j], a_im[i], accI[i][j]);
      // the next slab into the other buffer (last read before the previous barrier)
      if (s + 1 < nslab) store_slab(buf ^ 1);
      __syncthreads();
    }
  }

  // D's row (4 lk + r) is the output column, its column (lr) the output row
  if (p.splitk > 1) {
    cc* P = static_cast<cc*>(p.P) + (int64_t)split * p.M * p.N;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < 2; j++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int64_t m = m0 + wm0 + 16 * i + lr;
          const int64_t n = n0 + wn0 + 16 * j + 4 * lk + r;
          if (m < p.M && n < p.N) P[m + n * p.M] = make_float2(accR[i][j][r], accI[i][j][r]);
        }
    return;
  }
  cc* C = static_cast<cc*>(p.C);
  const cc* X = static_cast<const cc*>(p.X);
  const cc* Z = static_cast<const cc*>(p.Z);
  const cc* Rf = static_cast<const cc*>(p.R);
  const float al = (float)p.alpha, be = (float)p.beta, ga = (float)p.gamma;
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int64_t m = m0 + wm0 + 16 * i + lr;
        const int64_t n = n0 + wn0 + 16 * j + 4 * lk + r;
        if (m < p.M && n < p.N) {
          float vx = al * accR[i][j][r], vy = al * accI[i][j][r];
          if (X) {
            const cc x = X[m + n * p.ldx];
            vx += be * x.x;
            vy += be * x.y;
          }
          if (Z) {
            const cc z = Z[m + n * p.ldz];
            vx += ga * z.x;
            vy += ga * z.y;
          }
          if (Rf) {
            const cc rv = Rf[m + n * p.ldr];
            const float sc = (float)p.rs[n];
            vx += sc * rv.x;
            vy += sc * rv.y;
          }
          C[m + n * p.ldc] = make_float2(vx, vy);
        }
      }
}

// The split-K combination of a step: the partial tiles summed in split
// order, then the step's epilogue.
__global__ void __launch_bounds__(256) chebyshev_step_reduce_f16(ZGemmParams p) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p.M * p.N) return;
  const int64_t m = e % p.M, n = e / p.M;
  const cc* P = static_cast<const cc*>(p.P);
  float re = 0.f, im = 0.f;
#pragma unroll 8
  for (int s = 0; s < p.splitk; s++) {
    const cc v = P[(int64_t)s * p.M * p.N + e];
    re += v.x;
    im += v.y;
  }
  float vx = (float)p.alpha * re, vy = (float)p.alpha * im;
  if (p.X) {
    const cc x = static_cast<const cc*>(p.X)[m + n * p.ldx];
    vx += (float)p.beta * x.x;
    vy += (float)p.beta * x.y;
  }
  if (p.Z) {
    const cc z = static_cast<const cc*>(p.Z)[m + n * p.ldz];
    vx += (float)p.gamma * z.x;
    vy += (float)p.gamma * z.y;
  }
  if (p.R) {
    const cc rv = static_cast<const cc*>(p.R)[m + n * p.ldr];
    const float sc = (float)p.rs[n];
    vx += sc * rv.x;
    vy += sc * rv.y;
  }
  static_cast<cc*>(p.C)[m + n * p.ldc] = make_float2(vx, vy);
}

// out: the two FP16 planes of the n x n Hermitian A (column major, lda):
// plane row m = A(m, 0..n-1) = conj(column m of the stored A), zero to ld16.
__global__ void k_z2h_planes(const zc* A, int64_t lda, int64_t n, _Float16* out, int64_t ld16) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * ld16) return;
  const int64_t m = e / ld16, k = e % ld16;
  zc v = make_double2(0.0, 0.0);
  if (k < n) v = A[k + m * lda];
  out[m * ld16 + k] = (_Float16)v.x;
  out[n * ld16 + m * ld16 + k] = (_Float16)(-v.y);
}

}  // namespace

int64_t f16_plane_ld(int64_t n) { return cdiv(n, 64) * 64; }

void to_f16_planes(const zc* A, int64_t lda, int64_t n, void* out, hipStream_t st) {
  const int64_t ld16 = f16_plane_ld(n);
  const int64_t total = n * ld16;
  if (total == 0) return;
  hipLaunchKernelGGL(k_z2h_planes, dim3((unsigned)cdiv(total, 256)), dim3(256), 0, st, A, lda, n,
                     static_cast<_Float16*>(out), ld16);
  CHFSI_CHECK_LAUNCH();
}

void zgemm_f16_step(const GemmOp& g, const GemmWork& w, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return;
  if (g.opA != OP_N || g.opB != OP_N || g.flags || (g.batch > 1) || g.lda % 64 != 0 || g.lda < g.K ||
      g.ldb < g.K || (g.R && (!g.rs || g.ldr < g.M)))
    throw Error(ST_EINVAL, "FP16 step: op = N, batch 1, no flags, lda a multiple of 64 and >= K");
  ZGemmParams p{};
  p.M = g.M; p.N = g.N; p.K = g.K;
  p.A = g.A; p.lda = g.lda;
  p.B = g.B; p.ldb = g.ldb;
  p.C = g.C; p.ldc = g.ldc;
  p.X = g.X; p.ldx = g.ldx;
  p.Z = g.Z; p.ldz = g.ldz;
  p.alpha = g.alpha; p.beta = g.beta; p.gamma = g.gamma;
  p.R = g.R; p.ldr = g.ldr; p.rs = g.rs;
  p.tiles_m = (int)cdiv(g.M, HB);
  p.tiles_n = (int)cdiv(g.N, HB);
  const int64_t tiles = (int64_t)p.tiles_m * p.tiles_n;
  // K split: enough workgroups to fill the device several times over (four
  // per CU), chunks at least 256 deep, within the partial-tile scratch
  int64_t sk = g.splitk > 0 ? g.splitk : std::min<int64_t>(16, cdiv(1024, tiles));
  sk = std::max<int64_t>(1, std::min<int64_t>(sk, g.K / 256));
  const size_t cap = 2 * w.P_elems;  // complex FP32 elements
  while (sk > 1 && (!w.P || (size_t)sk * g.M * g.N > cap)) sk--;
  p.kchunk = cdiv(cdiv(g.K, sk), (int64_t)HK) * HK;
  p.splitk = (int)cdiv(g.K, p.kchunk);
  p.P = p.splitk > 1 ? (void*)w.P : nullptr;
  hipLaunchKernelGGL(chebyshev_step_f16, dim3((unsigned)tiles, (unsigned)p.splitk), dim3(HNT), 0, st, p);
  CHFSI_CHECK_LAUNCH();
  if (p.splitk > 1) {
    hipLaunchKernelGGL(chebyshev_step_reduce_f16, dim3((unsigned)cdiv(g.M * g.N, 256)), dim3(256), 0, st, p);
    CHFSI_CHECK_LAUNCH();
  }
}

}  // namespace chfsi
