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
// over a 128 x 64 output tile per workgroup of four waves (2 x 2, 64 x 32
// each as 4 x 2 fragments of 16 x 16), or 64 x 64 (32 x 32 per wave) for
// 65-160 columns (a 128 x 128 tile can be asked for), K in slabs of 32
// staged through LDS and double buffered; each complex product is four real
// products.  B is read as FP16 planes that the previous step's epilogue
// wrote beside its FP32 output (or, without them, as FP32 converted on the
// way into LDS).  As in
// the FP64 and FP32 steps, the product is formed transposed inside the
// matrix instruction (the B fragment first), so a wave's result lanes run
// down an output column.
#include <mutex>

#include "gemm.hpp"

namespace chfsi {

namespace {

typedef _Float16 h8v __attribute__((ext_vector_type(8)));

constexpr int HK = 32;          // slab depth (one matrix instruction per fragment pair and real product)
constexpr int HLD = HK + 8;     // LDS row stride in halves: 80 bytes, so 16 lanes' 16-byte reads hit distinct banks

__device__ __forceinline__ int64_t xcd_tile_h(int64_t bid, int64_t ntiles) {
  const int64_t full = (ntiles / 8) * 8;
  return bid < full ? (bid % 8) * (ntiles / 8) + bid / 8 : bid;
}

__device__ __forceinline__ f4v mfma_h(h8v a, h8v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// One step over a BM x BN output tile per workgroup of WM x WN waves, each
// wave (BM / WM) x (BN / WN) as 16 x 16 fragments.  LDS (dynamic):
// [buffer][re, im][row m][k] for A, then [buffer][re, im][column n][k] for B.
template <int BM, int BN, int WM, int WN, int MINB>
__global__ void __launch_bounds__(64 * WM * WN, MINB) chebyshev_step_f16(ZGemmParams p) {
  constexpr int NT = 64 * WM * WN;
  constexpr int MI = BM / (16 * WM), NJ = BN / (16 * WN);
  constexpr int AQ = BM * 4 / NT, BQ = BN * 4 / NT;  // rows / columns of a slab per thread
  static_assert(AQ >= 1 && BQ >= 1 && BM * 4 % NT == 0 && BN * 4 % NT == 0, "slab share");
  extern __shared__ __attribute__((aligned(16))) _Float16 hsm[];
  auto as_ = [&](int buf, int pl, int row) { return hsm + ((buf * 2 + pl) * BM + row) * HLD; };
  auto bs_ = [&](int buf, int pl, int col) { return hsm + 4 * BM * HLD + ((buf * 2 + pl) * BN + col) * HLD; };
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int wm0 = (wave % WM) * (BM / WM), wn0 = (wave / WM) * (BN / WN);

  const int64_t t = xcd_tile_h(blockIdx.x, (int64_t)p.tiles_m * p.tiles_n);
  const int64_t m0 = (t / p.tiles_n) * BM, n0 = (t % p.tiles_n) * BN;
  const int split = (int)blockIdx.y;
  const int64_t kbeg = (int64_t)split * p.kchunk;
  const int64_t kend = min(p.K, kbeg + p.kchunk);
  const int64_t nslab = kend > kbeg ? cdiv(kend - kbeg, (int64_t)HK) : 0;

  const _Float16* __restrict__ Are = static_cast<const _Float16*>(p.A);
  const _Float16* __restrict__ Aim = Are + p.M * p.lda;
  const cc* __restrict__ B = static_cast<const cc*>(p.B);
  const _Float16* __restrict__ B16 = static_cast<const _Float16*>(p.B16);

  // this thread's share of a slab: rows (A) / columns (B) tid / 4 + q NT / 4,
  // eight consecutive k from 8 (tid % 4)
  const int lrow = tid >> 2, lk8 = (tid & 3) * 8;
  uint4 ra_re[AQ], ra_im[AQ];
  h8v rb_re[BQ], rb_im[BQ];

  auto load_slab = [&](int64_t k0) {
    const int64_t k = k0 + lk8;
    // A: rows are zero-padded to lda (a multiple of 64) and chunk ends are
    // multiples of the slab depth, so only the row needs a check
#pragma unroll
    for (int q = 0; q < AQ; q++) {
      const int64_t gm = m0 + lrow + q * (NT / 4);
      if (gm < p.M) {
        ra_re[q] = *reinterpret_cast<const uint4*>(Are + gm * p.lda + k);
        ra_im[q] = *reinterpret_cast<const uint4*>(Aim + gm * p.lda + k);
      } else {
        ra_re[q] = make_uint4(0, 0, 0, 0);
        ra_im[q] = make_uint4(0, 0, 0, 0);
      }
    }
    if (B16) {
      // the previous step's FP16 copy: zero from row K on, so only the
      // column needs a check
#pragma unroll
      for (int q = 0; q < BQ; q++) {
        const int64_t gn = n0 + lrow + q * (NT / 4);
        if (gn < p.N) {
          rb_re[q] = *reinterpret_cast<const h8v*>(B16 + gn * p.ld16 + k);
          rb_im[q] = *reinterpret_cast<const h8v*>(B16 + p.pl16 + gn * p.ld16 + k);
        } else {
          rb_re[q] = h8v{};
          rb_im[q] = h8v{};
        }
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < BQ; q++) {
      const int64_t gn = n0 + lrow + q * (NT / 4);
      if (gn < p.N && k + 8 <= kend) {
        const cc* col = B + gn * p.ldb + k;
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const cc v = col[j];
          rb_re[q][j] = (_Float16)v.x;
          rb_im[q][j] = (_Float16)v.y;
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; j++) {
          cc v = make_float2(0.f, 0.f);
          if (gn < p.N && k + j < kend) v = B[gn * p.ldb + k + j];
          rb_re[q][j] = (_Float16)v.x;
          rb_im[q][j] = (_Float16)v.y;
        }
      }
    }
  };
  auto store_slab = [&](int buf) {
#pragma unroll
    for (int q = 0; q < AQ; q++) {
      *reinterpret_cast<uint4*>(as_(buf, 0, lrow + q * (NT / 4)) + lk8) = ra_re[q];
      *reinterpret_cast<uint4*>(as_(buf, 1, lrow + q * (NT / 4)) + lk8) = ra_im[q];
    }
#pragma unroll
    for (int q = 0; q < BQ; q++) {
      *reinterpret_cast<h8v*>(bs_(buf, 0, lrow + q * (NT / 4)) + lk8) = rb_re[q];
      *reinterpret_cast<h8v*>(bs_(buf, 1, lrow + q * (NT / 4)) + lk8) = rb_im[q];
    }
  };

  f4v accR[MI][NJ], accI[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; i++)
#pragma unroll
    for (int j = 0; j < NJ; j++) {
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
      h8v a_re[MI], a_im[MI], b_re[NJ], b_im[NJ], nb_im[NJ];
#pragma unroll
      for (int i = 0; i < MI; i++) {
        a_re[i] = *reinterpret_cast<const h8v*>(as_(buf, 0, wm0 + 16 * i + lr) + 8 * lk);
        a_im[i] = *reinterpret_cast<const h8v*>(as_(buf, 1, wm0 + 16 * i + lr) + 8 * lk);
      }
#pragma unroll
      for (int j = 0; j < NJ; j++) {
        b_re[j] = *reinterpret_cast<const h8v*>(bs_(buf, 0, wn0 + 16 * j + lr) + 8 * lk);
        b_im[j] = *reinterpret_cast<const h8v*>(bs_(buf, 1, wn0 + 16 * j + lr) + 8 * lk);
        nb_im[j] = -b_im[j];
      }
      // D[n][m] += B[k][n] A[m][k]: re = Br Ar - Bi Ai, im = Bi Ar + Br Ai,
      // issued type by type (dependent accumulations MI NJ instructions apart)
#pragma unroll
      for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < NJ; j++) accR[i][j] = mfma_h(b_re[j], a_re[i], accR[i][j]);
#pragma unroll
      for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < NJ; j++) accI[i][j] = mfma_h(b_im[j], a_re[i], accI[i][j]);
#pragma unroll
      for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < NJ; j++) accR[i][j] = mfma_h(nb_im[j], a_im[i], accR[i][j]);
#pragma unroll
      for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < NJ; j++) accI[i][j] = mfma_h(b_re[j], a_im[i], accI[i][j]);
      // the next slab into the other buffer (last read before the previous barrier)
      if (s + 1 < nslab) store_slab(buf ^ 1);
      __syncthreads();
    }
  }

  // D's row (4 lk + r) is the output column, its column (lr) the output row
  if (p.splitk > 1) {
    cc* P = static_cast<cc*>(p.P) + (int64_t)split * p.M * p.N;
#pragma unroll
    for (int i = 0; i < MI; i++)
#pragma unroll
      for (int j = 0; j < NJ; j++)
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
  _Float16* C16 = static_cast<_Float16*>(p.C16);
  const float al = (float)p.alpha, be = (float)p.beta, ga = (float)p.gamma;
#pragma unroll
  for (int i = 0; i < MI; i++)
#pragma unroll
    for (int j = 0; j < NJ; j++)
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
          if (C16) {
            C16[n * p.ld16 + m] = (_Float16)vx;
            C16[p.pl16 + n * p.ld16 + m] = (_Float16)vy;
          }
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
  if (p.C16) {
    _Float16* C16 = static_cast<_Float16*>(p.C16);
    C16[n * p.ld16 + m] = (_Float16)vx;
    C16[p.pl16 + n * p.ld16 + m] = (_Float16)vy;
  }
}

// FP16 planes of an m x ncols complex FP32 block (column n: re at
// out + n ld16, im pl16 further; rows m .. ld16 - 1 left as they are).
__global__ void k_c2h_cols(const cc* D, int64_t ldd, int64_t m, int64_t ncols, _Float16* out, int64_t ld16,
                           int64_t pl16) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * ncols) return;
  const int64_t i = e % m, j = e / m;
  const cc v = D[i + j * ldd];
  out[j * ld16 + i] = (_Float16)v.x;
  out[pl16 + j * ld16 + i] = (_Float16)v.y;
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

namespace {

template <int BM, int BN, int WM, int WN, int MINB>
void launch_f16(ZGemmParams& p, const GemmOp& g, const GemmWork& w, hipStream_t st) {
  constexpr size_t shm = (size_t)4 * (BM + BN) * HLD * sizeof(_Float16);
  static std::once_flag attr;
  std::call_once(attr, [&] {
    CHFSI_HIP(hipFuncSetAttribute((const void*)chebyshev_step_f16<BM, BN, WM, WN, MINB>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  });
  p.tiles_m = (int)cdiv(g.M, BM);
  p.tiles_n = (int)cdiv(g.N, BN);
  const int64_t tiles = (int64_t)p.tiles_m * p.tiles_n;
  // K split: enough workgroups to fill the device several times over,
  // chunks at least 256 deep, within the partial-tile scratch
  const int64_t want = BM * BN >= 128 * 128 ? 512 : 1024;
  int64_t sk = g.splitk > 0 ? g.splitk : std::min<int64_t>(16, cdiv(want, tiles));
  sk = std::max<int64_t>(1, std::min<int64_t>(sk, g.K / 256));
  const size_t cap = 2 * w.P_elems;  // complex FP32 elements
  while (sk > 1 && (!w.P || (size_t)sk * g.M * g.N > cap)) sk--;
  p.kchunk = cdiv(cdiv(g.K, sk), (int64_t)HK) * HK;
  p.splitk = (int)cdiv(g.K, p.kchunk);
  p.P = p.splitk > 1 ? (void*)w.P : nullptr;
  hipLaunchKernelGGL((chebyshev_step_f16<BM, BN, WM, WN, MINB>), dim3((unsigned)tiles, (unsigned)p.splitk),
                     dim3(64 * WM * WN), shm, st, p);
  CHFSI_CHECK_LAUNCH();
}

}  // namespace

void to_f16_cols(const cc* D, int64_t ldd, int64_t m, int64_t ncols, void* out, int64_t ld16, int64_t pl16,
                 hipStream_t st) {
  if (m * ncols == 0) return;
  hipLaunchKernelGGL(k_c2h_cols, dim3((unsigned)cdiv(m * ncols, 256)), dim3(256), 0, st, D, ldd, m, ncols,
                     static_cast<_Float16*>(out), ld16, pl16);
  CHFSI_CHECK_LAUNCH();
}

void zgemm_f16_step(const GemmOp& g, const GemmWork& w, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return;
  if (g.opA != OP_N || g.opB != OP_N || g.flags || (g.batch > 1) || g.lda % 64 != 0 || g.lda < g.K ||
      g.ldb < g.K || (g.R && (!g.rs || g.ldr < g.M)) ||
      ((g.B16 || g.C16) && (g.ld16 % 64 != 0 || g.ld16 < g.K || g.ld16 < g.M || g.pl16 < g.N * g.ld16)))
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
  p.B16 = g.B16; p.C16 = g.C16; p.ld16 = g.ld16; p.pl16 = g.pl16;
  // tile shape (the FP64 / FP32 numbering: 1 = 64 x 64, 4 = 128 x 64,
  // 6 = 128 x 128); automatic: 64 x 64 for 65-160 columns (3-9 % faster
  // there at n = 4000 and 10000), else 128 x 64 (the fastest or within 4 %
  // at the other widths measured, 48 to 600; 128 x 128 holds one workgroup
  // per CU and trails by up to 35 % at narrow widths)
  const int cfg = g.cfg != 0 ? g.cfg : (g.N > 64 && g.N <= 160 ? 1 : 4);
  switch (cfg) {
    case 1: launch_f16<64, 64, 2, 2, 4>(p, g, w, st); break;    // 40 KB of LDS: four per CU
    case 4: launch_f16<128, 64, 2, 2, 2>(p, g, w, st); break;   // 60 KB: two per CU
    case 6: launch_f16<128, 128, 2, 4, 2>(p, g, w, st); break;  // 80 KB: two per CU
    default: throw Error(ST_EINVAL, "FP16 step: tile configuration 0, 1, 4 or 6");
  }
  if (p.splitk > 1) {
    hipLaunchKernelGGL(chebyshev_step_reduce_f16, dim3((unsigned)cdiv(g.M * g.N, 256)), dim3(256), 0, st, p);
    CHFSI_CHECK_LAUNCH();
  }
}

}  // namespace chfsi
