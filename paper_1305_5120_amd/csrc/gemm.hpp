// Internal interface of the complex GEMM kernels (FP64 and FP32).
#pragma once

#include <algorithm>

#include "common.hpp"

namespace chfsi {

enum { OP_N = 0, OP_C = 1 };

// Structure flags.  TRI_*: op(A) / op(B) is triangular with explicit zeros
// stored in the other triangle, so each tile may skip the K range that only
// meets zeros.  OUT_LOWER: only tiles touching the lower triangle of the
// output are computed (the rest of the output is left untouched).
enum {
  GEMM_TRI_A_LOWER = 1,  // op(A)[m,k] = 0 for k > m
  GEMM_TRI_A_UPPER = 2,  // op(A)[m,k] = 0 for k < m
  GEMM_TRI_B_LOWER = 4,  // op(B)[k,n] = 0 for k < n
  GEMM_TRI_B_UPPER = 8,  // op(B)[k,n] = 0 for k > n
  GEMM_OUT_LOWER = 16,
};

enum { PREC_F64 = 0, PREC_F32 = 1 };

// out = alpha * op(A) op(B) + beta * X + gamma * Z, op(A) M x K, op(B) K x N.
// X / Z may be null; out may alias X or Z (each element is read and written
// by the same thread) but must not alias A or B.  Elements are complex FP64
// (zc) or, with prec = PREC_F32 (op = N on both sides only), complex FP32
// (cc) with FP32 accumulation.
struct GemmOp {
  int prec = PREC_F64;
  int opA = OP_N, opB = OP_N;
  int64_t M = 0, N = 0, K = 0;
  const void* A = nullptr; int64_t lda = 0, sA = 0;
  const void* B = nullptr; int64_t ldb = 0, sB = 0;
  void* C = nullptr; int64_t ldc = 0, sC = 0;
  const void* X = nullptr; int64_t ldx = 0, sX = 0;
  const void* Z = nullptr; int64_t ldz = 0, sZ = 0;
  double alpha = 1.0, beta = 0.0, gamma = 0.0;
  int flags = 0;
  int batch = 1;            // strided batch count (s* are the strides)
  bool allow_splitk = true;
  bool filter_step = false;  // launch under the Chebyshev-step kernel symbol
  int cfg = 0;              // tile configuration (0: chosen automatically)
  int splitk = 0;           // K split (0: chosen automatically, 1: none)
  // FP32 only, batch 1: out(:, j) += rs[j] R(:, j) (R complex FP32, M x N
  // with leading dimension ldr; rs device FP64, N entries), the forcing term
  // of the filter's Ritz-residual recurrence
  const void* R = nullptr; int64_t ldr = 0;
  const double* rs = nullptr;
  // FP16 steps only: B also as FP16 planes (column n holding its k
  // consecutively: re at B16 + n ld16, im pl16 halves further; zero from
  // row K to ld16), and C also written there (C16, same layout), the next
  // step's B; null: B read as FP32, no FP16 copy of C
  const void* B16 = nullptr; void* C16 = nullptr;
  int64_t ld16 = 0, pl16 = 0;
};

// Scratch for split-K partial tiles (P_elems complex FP64 elements; an FP32
// product uses the same bytes as twice as many complex FP32 elements).
struct GemmWork {
  zc* P = nullptr;
  size_t P_elems = 0;
};

struct ZGemmParams {
  int64_t M, N, K;
  const void* A; int64_t lda, sA;
  const void* B; int64_t ldb, sB;
  void* C; int64_t ldc, sC;
  const void* X; int64_t ldx, sX;
  const void* Z; int64_t ldz, sZ;
  double alpha, beta, gamma;
  int flags;
  int splitk;
  int64_t kchunk;
  void* P;
  int tiles_m, tiles_n;
  const void* R; int64_t ldr;  // FP32 only: out(:, j) += rs[j] R(:, j) (null: none)
  const double* rs;
  const void* B16; void* C16;  // FP16 steps only: FP16 planes of B and of the output
  int64_t ld16, pl16;
};

void zgemm(const GemmOp& g, const GemmWork& w, hipStream_t st);
void zgemm_choose(const GemmOp& g, int64_t P_elems, int& cfg, int& splitk);
int zgemm_num_configs();
// Tile shape (BM x BN) of configuration cfg; -1 if cfg is not a tile shape.
int zgemm_tile_shape(int cfg, int* bm, int* bn);
// One grouped filter step over G problems in precision prec: gp (device, G
// params with M, N, K, pointers, scalars and tiles_m / tiles_n filled,
// splitk = 1, kchunk = K), tile0 (device, G + 1 prefix of tiles_m * tiles_n),
// ctr (device, 8 ints, zero at launch: the XCDs' tile counters).
// Persistent grid of `grid` workgroups (multiple of 8).
void zgemm_grouped_filter_step(int prec, int cfg, const ZGemmParams* gp, const int64_t* tile0, int G, int* ctr,
                               int grid, hipStream_t st);
// The split-K combination of one grouped step: elem0 (device, G + 1 prefix
// of M * N over the problems whose params have splitk > 1, 0 elements for
// the others); grid-stride launch of `grid` workgroups.  The problems' split
// work items are counted in tile0 as tiles_m * tiles_n * splitk, with
// kchunk the K range of one split.
void zgemm_grouped_reduce(int prec, const ZGemmParams* gp, const int64_t* elem0, int G, int grid, hipStream_t st);
// The FP16 degree step (precision 3 of the solver): A in two FP16 planes
// made by to_f16_planes (row length f16_plane_ld(n), zero padded), B, X, Z,
// R and C complex FP32; op = N, batch 1, no flags; splitk 0 = automatic.
int64_t f16_plane_ld(int64_t n);
void to_f16_planes(const zc* A, int64_t lda, int64_t n, void* out, hipStream_t st);
void zgemm_f16_step(const GemmOp& g, const GemmWork& w, hipStream_t st);
// The FP16 planes (B16 layout above) of an m x ncols complex FP32 block.
void to_f16_cols(const cc* D, int64_t ldd, int64_t m, int64_t ncols, void* out, int64_t ld16, int64_t pl16,
                 hipStream_t st);
// K slab depth of a tile configuration (0 if cfg is not one).
int zgemm_config_bk(int cfg);
// Whether cfg can run the grouped step; the grid that fills the device with it.
bool zgemm_grouped_config_ok(int cfg);
int zgemm_grouped_grid(int prec, int cfg);

}  // namespace chfsi
