// Solver engine and C ABI of the ChFSI library.
//
// Host-side orchestration of Algorithm 1 (arXiv 1305.5120): every numerical
// step runs in this library's kernels (zgemm.hip, kernels.hip) on the
// context's stream; the host only sequences launches, reads back the k_a Ritz
// values and residual norms once per outer iteration and takes the locking
// decision.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdio>
#include <cstdlib>

#include "../../include/chfsi.h"
#include "gemm.hpp"
#include "kernels.hpp"

using namespace chfsi;

namespace {

// Named host ranges around the solver's phases, for profilers that record
// ROCTX markers (rocprofv3 --marker-trace); without one they cost a call.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// Diagnostics on stderr, from the environment variable CHFSI_LOG: 1 = one
// line per solve (sizes, iterations, phase times, residual), 2 = also one
// line per outer iteration (locked count, active width, precision split,
// filter interval, first active residual).
int log_level() {
  static const int level = [] {
    const char* e = std::getenv("CHFSI_LOG");
    return e ? std::atoi(e) : 0;
  }();
  return level;
}

struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void ensure(size_t b) {
    if (bytes >= b) return;
    if (p) CHFSI_HIP(hipFree(p));
    p = nullptr;
    bytes = 0;
    if (b == 0) return;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw Error(ST_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed: " + hipGetErrorString(e));
    }
    bytes = b;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  zc* z() const { return static_cast<zc*>(p); }
  double* d() const { return static_cast<double*>(p); }
  int* i() const { return static_cast<int*>(p); }
};

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
};

// Columns of split-K partial tiles a context keeps for a block of k columns
// (times n elements): four splits of the whole block, and up to eight for
// narrow blocks, where the filter's products split K eight ways.
size_t splitk_columns(int64_t k) {
  return std::max((size_t)4 * k, std::min((size_t)8 * k, (size_t)2560));
}

// Block sizes of a solve: 1 <= nev, nev + nex <= n, and at least one extra
// column unless the block is the whole space: the filter damps [a, b] with
// a the largest Ritz value of the block, which must not be a wanted one (with
// nex = 0 the nev-th wanted value sits on the damped interval's edge and its
// convergence stalls).
bool block_sizes_ok(int64_t n, int64_t nev, int64_t nex) {
  return nev >= 1 && nex >= 0 && nev + nex <= n && (nex >= 1 || nev == n);
}
constexpr const char* BLOCK_SIZES_RULE = "need 1 <= nev, nev + nex <= n and nex >= 1 unless nev = n";

// Coefficients of the m degree steps of the scaled Chebyshev filter
// (eq. (2) on (A - cI)/e, normalized at a0): step i computes
//   Y_{i+1} = alpha_i A Y_i + beta_i Y_i + gamma_i Y_{i-1}   (gamma_0 = 0).
struct ChebStep {
  double alpha, beta, gamma;
};

std::vector<ChebStep> cheb_schedule(int m, double a, double b, double a0) {
  std::vector<ChebStep> out(m);
  const double e = (b - a) / 2.0, c = (b + a) / 2.0;
  const double sigma1 = e / (a0 - c);
  const double tau = 2.0 / sigma1;
  const double al1 = sigma1 / e;
  out[0] = {al1, -al1 * c, 0.0};
  double sigma = sigma1;
  for (int i = 1; i < m; i++) {
    const double sn = 1.0 / (tau - sigma);
    const double al = 2.0 * sn / e;
    out[i] = {al, -al * c, -sigma * sn};
    sigma = sn;
  }
  return out;
}

}  // namespace

struct chfsi_ctx_s {
  int64_t n = 0;
  chfsi_opts opts{};
  hipStream_t st = nullptr;
  std::string err;

  // n x n: standard form, Cholesky factor, its inverse, work; FP32 copy of A
  DBuf A, L, Linv, W, A32;
  // FP16 planes of A (precision 3: two planes of n rows, f16_plane_ld(n) halves each)
  // and of the residual part's two iterates (each two planes of k columns)
  DBuf A16, D16;
  // FP32 filter blocks (mixed precision); the FP32 filter on the Ritz
  // residual: its forcing R (n x k, FP32) and the scalar recurrence's table
  DBuf Y32, Y32b, R32, ctab;
  bool have_factors = false;
  // n x k blocks
  DBuf Y, Yb, F, Qb, Wk, Wz;
  int64_t kcap = 0;
  int64_t nk_n = 0;  // n the n x k blocks were sized for
  // k x k and small
  DBuf G, Z, Z2, G2, Ztmp, mu, rho, rank, norms, flags;
  DBuf P;  // split-K partial tiles
  size_t P_elems = 0;
  // Householder
  DBuf hpart, htop, tau, Tall, gram, Vp, Wt, W2;
  // Lanczos
  DBuf LV, Lw, Lh, Lab, mvpart, Tsm, Tz, Tz2, Tw, npart;
  // sparse Jacobi schedules
  DBuf jint, jrot, bjv;
  // eigenvector refinement: six k x k blocks, Rayleigh quotients, max correction
  DBuf rf, rfl, rfc;
  // host staging (pinned)
  double* hbuf = nullptr;
  size_t hbuf_elems = 0;
  double* htab = nullptr;  // the Ritz-residual filter's table on its way up
  size_t htab_elems = 0;

  // warm state (Y holds the block)
  bool warm_valid = false;
  int64_t warm_k = 0;
  double warm_a0 = 0, warm_a = 0;

  // filter timing and work, per precision (0 FP64, 1 FP32)
  std::vector<EventPair> fev[2];  // per precision
  double filt_kernel_s[2] = {0, 0};
  int filt_launches[2] = {0, 0};
  double filt_flops[2] = {0, 0};
  bool filt_pending[2] = {false, false};  // events recorded since the last collection
  void reset_filter_stats() {
    for (int i = 0; i < 2; i++) {
      filt_kernel_s[i] = 0;
      filt_launches[i] = 0;
      filt_flops[i] = 0;
    }
  }

  // Split scratch the products may use: the part sized for the current
  // problem (n, k), not all the buffer has grown to, so that the splits
  // chosen - and the rounding of the results - do not depend on the sizes
  // a context served before (the serving loop reuses contexts across sizes).
  // Entry points that size the scratch for their own product widen it.
  size_t P_cap = 0;
  GemmWork gw() const { return GemmWork{P.z(), std::min(P_elems, P_cap)}; }
  static size_t split_scratch_elems(int64_t n, int64_t k, int filter_splitk) {
    return 8 * (size_t)k * k + (size_t)n * std::max((size_t)filter_splitk * k, splitk_columns(k)) + ((size_t)1 << 16);
  }


  void ensure_host(size_t elems) {
    if (hbuf_elems >= elems) return;
    if (hbuf) {
      CHFSI_HIP(hipStreamSynchronize(st));  // no copy may still target the old buffer
      (void)hipHostFree(hbuf);
    }
    hbuf = nullptr;
    hbuf_elems = 0;
    CHFSI_HIP(hipHostMalloc((void**)&hbuf, elems * sizeof(double), hipHostMallocDefault));
    hbuf_elems = elems;
  }

  void ensure_htab(size_t elems) {
    if (htab_elems >= elems) return;
    if (htab) {
      CHFSI_HIP(hipStreamSynchronize(st));
      (void)hipHostFree(htab);
    }
    htab = nullptr;
    htab_elems = 0;
    CHFSI_HIP(hipHostMalloc((void**)&htab, elems * sizeof(double), hipHostMallocDefault));
    htab_elems = elems;
  }

  void ensure_nn() {
    const size_t b = (size_t)n * n * sizeof(zc);
    A.ensure(b);
    L.ensure(b);
    Linv.ensure(b);
    W.ensure(b);
  }

  void ensure_k(int64_t k) {
    P_cap = split_scratch_elems(n, k, opts.filter_splitk);
    if (k <= kcap && Y.p && n <= nk_n) return;
    const int64_t kk = std::max<int64_t>(k, kcap);
    // keep the warm block across growth
    DBuf oldY;
    if (warm_valid && Y.p) {
      oldY.ensure((size_t)n * warm_k * sizeof(zc));
      CHFSI_HIP(hipMemcpyAsync(oldY.p, Y.p, (size_t)n * warm_k * sizeof(zc), hipMemcpyDeviceToDevice, st));
      CHFSI_HIP(hipStreamSynchronize(st));
    }
    const size_t nk = (size_t)n * kk * sizeof(zc);
    for (DBuf* b : {&Y, &Yb, &F, &Qb, &Wk, &Wz}) {
      b->release();
      b->ensure(nk);
    }
    const size_t kk2 = (size_t)kk * kk * sizeof(zc);
    for (DBuf* b : {&G, &Z, &Z2, &G2, &Ztmp}) {
      b->release();
      b->ensure(kk2);
    }
    rf.release(); rf.ensure((size_t)6 * kk * kk * sizeof(zc));
    rfl.release(); rfl.ensure((size_t)kk * sizeof(double));
    mu.release(); mu.ensure((size_t)kk * sizeof(double));
    rho.release(); rho.ensure((size_t)kk * sizeof(double));
    rank.release(); rank.ensure((size_t)kk * sizeof(int));
    P_elems = split_scratch_elems(n, kk, opts.filter_splitk);
    P.release();
    P.ensure(P_elems * sizeof(zc));
    const int64_t npan = cdiv(kk, HH_NB);
    hpart.release(); hpart.ensure((size_t)2 * 256 * HH_NB * sizeof(zc));
    htop.release(); htop.ensure((size_t)2 * HH_NB * sizeof(zc));
    tau.release(); tau.ensure((size_t)kk * sizeof(zc));
    Tall.release(); Tall.ensure((size_t)npan * HH_NB * HH_NB * sizeof(zc));
    gram.release(); gram.ensure((size_t)HH_NB * HH_NB * sizeof(zc));
    Vp.release(); Vp.ensure((size_t)n * HH_NB * sizeof(zc));
    Wt.release(); Wt.ensure((size_t)HH_NB * kk * sizeof(zc));
    W2.release(); W2.ensure((size_t)HH_NB * kk * sizeof(zc));
    ensure_host(4 * (size_t)kk + 256);
    if (oldY.p) {
      CHFSI_HIP(hipMemcpyAsync(Y.p, oldY.p, (size_t)n * warm_k * sizeof(zc), hipMemcpyDeviceToDevice, st));
      CHFSI_HIP(hipStreamSynchronize(st));
      oldY.release();
    }
    kcap = kk;
    nk_n = n;
  }

  // Take problems of size n_new with the same buffers: every buffer is
  // checked against the size it needs before use and only grows, so a
  // context made for a larger n serves smaller ones without new
  // allocations.  The factor and the kept block belong to the old size and
  // are dropped.
  void resize(int64_t n_new) {
    if (n_new == n) return;
    n = n_new;
    have_factors = false;
    warm_valid = false;
  }

  void ensure_small() {
    norms.ensure(8 * sizeof(double));
    rfc.ensure(4 * sizeof(unsigned long long));
    flags.ensure(8 * sizeof(int));
    const int steps = std::max(1, opts.lanczos_steps);
    LV.ensure((size_t)n * (steps + 1) * sizeof(zc));
    Lw.ensure((size_t)n * sizeof(zc));
    Lh.ensure((size_t)(steps + 2) * sizeof(zc));
    Lab.ensure((size_t)2 * (steps + 2) * sizeof(double));
    mvpart.ensure((size_t)32 * n * sizeof(zc));
    Tsm.ensure((size_t)JACOBI_LDS_MAX * JACOBI_LDS_MAX * sizeof(zc));
    Tz.ensure((size_t)JACOBI_LDS_MAX * JACOBI_LDS_MAX * sizeof(zc));
    Tz2.ensure((size_t)JACOBI_LDS_MAX * JACOBI_LDS_MAX * sizeof(zc));
    npart.ensure(1024 * sizeof(double));
    Tw.ensure((size_t)JACOBI_LDS_MAX * 2 * sizeof(double) + 64);
    ensure_host(2 * JACOBI_LDS_MAX * JACOBI_LDS_MAX + 512);
  }

  void sync() { CHFSI_HIP(hipStreamSynchronize(st)); }

  void free_all() {
    for (DBuf* b : {&A32, &A16, &D16, &Y32, &Y32b, &R32, &ctab, &A, &L, &Linv, &W, &Y, &Yb, &F, &Qb, &Wk, &Wz, &G, &Z, &Z2, &G2, &Ztmp, &mu, &rho, &rank, &norms,
                    &flags, &P, &hpart, &htop, &tau, &Tall, &gram, &Vp, &Wt, &W2, &LV, &Lw, &Lh, &Lab, &mvpart, &Tsm,
                    &Tz, &Tz2, &Tw, &npart, &jint, &jrot, &bjv, &rf, &rfl, &rfc})
      b->release();
    if (hbuf) (void)hipHostFree(hbuf);
    hbuf = nullptr;
    if (htab) (void)hipHostFree(htab);
    htab = nullptr;
    htab_elems = 0;
    for (auto& v : fev) {
      for (auto& e : v) {
        if (e.a) (void)hipEventDestroy(e.a);
        if (e.b) (void)hipEventDestroy(e.b);
      }
      v.clear();
    }
  }

  // ------------------------------------------------------------------------
  // GEMM helper
  // ------------------------------------------------------------------------
  void gemm(int opA, int opB, int64_t M, int64_t N, int64_t K, double alpha, const zc* Ap, int64_t lda, const zc* Bp,
            int64_t ldb, zc* Cp, int64_t ldc, double beta = 0.0, const zc* X = nullptr, int64_t ldx = 0, double gamma = 0.0,
            const zc* Zp = nullptr, int64_t ldz = 0, int flags_ = 0, bool splitk = true, bool filter_step = false,
            int cfg = 0, int nsplit = 0) {
    GemmOp g;
    g.cfg = cfg;
    g.splitk = nsplit;
    g.filter_step = filter_step;
    g.opA = opA; g.opB = opB; g.M = M; g.N = N; g.K = K;
    g.A = Ap; g.lda = lda; g.B = Bp; g.ldb = ldb; g.C = Cp; g.ldc = ldc;
    g.X = X; g.ldx = ldx; g.Z = Zp; g.ldz = ldz;
    g.alpha = alpha; g.beta = beta; g.gamma = gamma;
    g.flags = flags_;
    g.allow_splitk = splitk;
    zgemm(g, gw(), st);
  }

  // ------------------------------------------------------------------------
  // Reduction to standard form
  // ------------------------------------------------------------------------
  // Blocked Cholesky of the m x m Hermitian matrix src (lower triangle read)
  // into Lb (strict upper triangle zero) and Lib = Lb^{-1}; Wb is m x m work;
  // all with leading dimension ld.  Returns 0, or the 1-based column of the
  // first pivot that is not positive (then Lb / Lib are incomplete).
  // Blocked Cholesky of the m x m Hermitian matrix whose lower triangle src
  // holds (the upper triangle is not read): Lb = L, Lib = L^{-1} (both with
  // zero strict upper triangles), Wb scratch.  With info_d null the host
  // waits and the first non-positive pivot's column + 1 is returned (0 when
  // positive definite).  With info_d (device int) nothing waits: the column
  // + 1 lands there (INT_MAX when positive definite) and Lb, Lib are
  // meaningless when it is not; the caller reads it when convenient.
  int chol_factor(int64_t m, const zc* src, int64_t lds, zc* Wb, zc* Lb, zc* Lib, int64_t ld, int* info_d = nullptr) {
    const int64_t NB = CHOL_NB;
    int* info = info_d ? info_d : flags.i();
    fill_i32(info, 1, INT_MAX, st);
    if (m <= NB) {
      // one diagonal block: factor and inverse in one launch, straight from
      // src (no trailing updates touch it); the kernel writes the zeros
      chol_diag(src, lds, Lb, ld, Lib, ld, 0, m, info, st);
    } else {
      copy2d(src, lds, Wb, ld, m, m, st);
      // two levels: outer blocks of CHOL_NB_OUTER columns, whose trailing
      // updates are deep products (rank 256 instead of 64); each outer
      // diagonal block is factored with the 64-column diagonal kernel and
      // its own inner updates, and its inverse completed, before the outer
      // panel below it is solved with that inverse
      const int64_t NBO = m > CHOL_NB_OUTER ? CHOL_NB_OUTER : m;
      for (int64_t b0 = 0; b0 < m; b0 += NBO) {
        const int64_t bn = std::min(NBO, m - b0), r = m - b0 - bn;
        for (int64_t j0 = b0; j0 < b0 + bn; j0 += NB) {
          const int64_t nb = std::min(NB, b0 + bn - j0), ri = b0 + bn - j0 - nb;
          chol_diag(Wb, ld, Lb, ld, Lib, ld, j0, nb, info, st);
          if (ri > 0) chol_update(Wb, Lb, Lib, ld, j0, nb, ri);
        }
        // the products below read the triangular blocks in whole tiles: the
        // block's strict upper triangle must hold zeros (the diagonal kernel
        // writes them inside its 64 x 64 blocks, nothing writes the rest)
        zero_strict_upper(Lib + b0 + b0 * ld, ld, bn, st);
        inverse_doubling(Lb, Lib, ld, b0, bn, NB, Wb);
        if (r > 0) chol_update(Wb, Lb, Lib, ld, b0, bn, r);
      }
      zero_strict_upper(Lb, ld, m, st);
    }
    if (!info_d) {
      CHFSI_HIP(hipMemcpyAsync(hbuf, flags.p, sizeof(int), hipMemcpyDeviceToHost, st));
      sync();
      int hinfo;
      std::memcpy(&hinfo, hbuf, sizeof(int));
      if (hinfo != INT_MAX) return hinfo;
    }
    if (m <= NB) return 0;
    // the diagonal blocks of Lib (CHOL_NB_OUTER wide) are complete: the rest
    // by recursive doubling from there
    inverse_doubling(Lb, Lib, ld, 0, m, std::min<int64_t>(m, CHOL_NB_OUTER), Wb);
    zero_strict_upper(Lib, ld, m, st);
    return 0;
  }

  // Below a factored diagonal block (columns j0 .. j0 + nb, inverse in Lib):
  // the panel L21 = W21 L11^{-H} of the next r rows, then W22 -= L21 L21^H
  // (lower tiles) over those rows.
  void chol_update(zc* Wb, zc* Lb, const zc* Lib, int64_t ld, int64_t j0, int64_t nb, int64_t r) {
    gemm(OP_N, OP_C, r, nb, nb, 1.0, Wb + (j0 + nb) + j0 * ld, ld, Lib + j0 + j0 * ld, ld, Lb + (j0 + nb) + j0 * ld, ld,
         0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_TRI_B_UPPER, false);
    zc* W22 = Wb + (j0 + nb) + (j0 + nb) * ld;
    const zc* L21 = Lb + (j0 + nb) + j0 * ld;
    gemm(OP_N, OP_C, r, r, nb, -1.0, L21, ld, L21, ld, W22, ld, 1.0, W22, ld, 0.0, nullptr, 0, GEMM_OUT_LOWER, false);
  }

  // Lib over rows / columns b0 .. b0 + bn from its complete diagonal blocks
  // of s0 columns (aligned at b0) by recursive doubling,
  //   inv([[L11, 0], [L21, L22]]) = [[X11, 0], [-X22 L21 X11, X22]];
  // T (ld) is work.
  void inverse_doubling(const zc* Lb, zc* Lib, int64_t ld, int64_t b0, int64_t bn, int64_t s0, zc* T) {
    for (int64_t s = s0; s < bn; s *= 2) {
      for (int64_t i0 = b0; i0 + s < b0 + bn; i0 += 2 * s) {
        const int64_t b = std::min(s, b0 + bn - i0 - s);
        const zc* L21 = Lb + (i0 + s) + i0 * ld;
        const zc* X11 = Lib + i0 + i0 * ld;
        const zc* X22 = Lib + (i0 + s) + (i0 + s) * ld;
        gemm(OP_N, OP_N, b, s, s, 1.0, L21, ld, X11, ld, T, ld, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_TRI_B_LOWER);
        gemm(OP_N, OP_N, b, s, b, -1.0, X22, ld, T, ld, Lib + (i0 + s) + i0 * ld, ld, 0.0, nullptr, 0, 0.0, nullptr, 0,
             GEMM_TRI_A_LOWER);
      }
    }
  }

  void cholesky(const zc* S, int64_t lds) {
    const int info = chol_factor(n, S, lds, W.z(), L.z(), Linv.z(), n);
    if (info) {
      have_factors = false;
      throw Error(ST_ENOTPD, "S is not positive definite: pivot of column " + std::to_string(info - 1) + " is not positive");
    }
    have_factors = true;
  }

  // keep_warm: a kept warm block (standard form of the factor being
  // replaced) is carried over to the new factor through the generalized
  // space, X = L_old^{-H} Y, Y = L_new^H X (Sec. 2: the previous problem's
  // eigenvectors start the next one; with a new overlap matrix they are the
  // generalized vectors that carry over).  Without keep_warm, or when the new
  // factorization fails, the kept block is dropped: it would no longer match
  // the context's factor.
  void reduce(const zc* H, int64_t ldh, const zc* S, int64_t lds, bool keep_warm = true) {
    ensure_nn();
    ensure_small();
    if (warm_valid && !have_factors) warm_valid = false;
    if (S) {
      const bool remap = keep_warm && warm_valid && Y.p && warm_k > 0 && warm_k <= kcap;
      if (remap)
        gemm(OP_C, OP_N, n, warm_k, n, 1.0, Linv.z(), n, Y.z(), n, F.z(), n, 0.0, nullptr, 0, 0.0, nullptr, 0,
             GEMM_TRI_A_UPPER);
      warm_valid = false;  // until the block is in the new factor's standard form
      cholesky(S, lds);
      if (remap) {
        gemm(OP_C, OP_N, n, warm_k, n, 1.0, L.z(), n, F.z(), n, Y.z(), n, 0.0, nullptr, 0, 0.0, nullptr, 0,
             GEMM_TRI_A_UPPER);
        warm_valid = true;
      }
    } else if (!have_factors) {
      throw Error(ST_EINVAL, "no cached factor of S: pass S");
    }
    // A = Linv H Linv^H; A is Hermitian, so the second product forms only
    // the tiles that touch its lower triangle and the upper one is mirrored
    gemm(OP_N, OP_N, n, n, n, 1.0, Linv.z(), n, H, ldh, W.z(), n, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_TRI_A_LOWER);
    gemm(OP_N, OP_C, n, n, n, 1.0, W.z(), n, Linv.z(), n, A.z(), n, 0.0, nullptr, 0, 0.0, nullptr, 0,
         GEMM_TRI_B_UPPER | GEMM_OUT_LOWER);
    hermitian_from_lower(A.z(), n, n, st);
  }

  // ------------------------------------------------------------------------
  // Hermitian eigensolver (Jacobi) into w (device, ascending), Zo (device)
  // ------------------------------------------------------------------------
  // tau > 0: couplings |G(p,q)| <= tau count as converged (the solver passes
  // a value far below its lock scale: such couplings change Ritz vectors by
  // less than their residual tolerance); tau = 0 iterates to working accuracy.
  void eigh(const zc* Gp, int64_t ldg, int64_t k, double* w, zc* Zo, int64_t ldz, double tau = 0.0) {
    if (k <= JACOBI_LDS_MAX) {
      // nearly diagonal (the projected matrices of warm iterations): the
      // refinement's few small products beat the sweeps of one workgroup;
      // otherwise Jacobi in one workgroup
      if (k >= SMALL_REFINE_MIN) {
        jacobi_init(Gp, ldg, k, G2.z(), Ztmp.z(), st);
        if (refine(G2.z(), nullptr, k, w, Zo, ldz, tau)) return;
      }
      jacobi_small(Gp, ldg, k, w, Zo, ldz, Ztmp.z(), nullptr, st, tau);
      return;
    }
    // Larger k.  Each pass: if the matrix is nearly diagonal, refinement
    // finishes (refine); else, if the pairs that block the refinement (a
    // coupling above REF_ETA times the gap of their diagonal entries) are
    // few, a sparse sweep rotates only those; else a sparse sweep over all
    // significant couplings (|g|^2 > 1e-34 ||G||_F^2) when they are few, or
    // a dense sweep in a block ordering (blocks of 16 indices paired
    // round-robin, each pair's 32 x 32 subproblem swept in LDS).  Sparse
    // sweeps group their pairs into disjoint rounds.
    zc *g0 = G2.z(), *z0 = Ztmp.z();
    jacobi_init(Gp, ldg, k, g0, z0, st);
    double* nr = norms.d();
    jacobi_norms(g0, k, npart.d(), nr, st);  // nr[0] = off, nr[1] = all (fro2)
    const double THR = 1e-34;
    const int64_t max_sparse = 8 * k;
    const int max_rounds = 64;
    const size_t ints = (size_t)2 * k + 2 * max_sparse + (size_t)max_rounds * k + 2 * max_sparse;
    jint.ensure(ints * sizeof(int));
    jrot.ensure((size_t)(k / 2 + 1) * jacobi_rot_bytes());
    ensure_host(ints / 2 + 16);
    int* counts = jint.i();
    int* offsets = counts + k;
    int* pairs = offsets + k;
    int* rounds_d = pairs + 2 * max_sparse;
    // One sparse sweep over the pairs selected by (thr, ratio); returns the
    // number of selected pairs, or -1 (nothing applied) when they are too
    // many or cannot be packed into max_rounds disjoint rounds.
    auto sparse_sweep = [&](double ratio) -> int64_t {
      jacobi_count(g0, k, nr + 1, THR, tau, ratio, counts, st);
      CHFSI_HIP(hipMemcpyAsync(hbuf, counts, k * sizeof(int), hipMemcpyDeviceToHost, st));
      sync();
      const int* hc = reinterpret_cast<const int*>(hbuf);
      int64_t total = 0;
      std::vector<int> off(k);
      for (int64_t j = 0; j < k; j++) {
        off[j] = (int)total;
        total += hc[j];
      }
      if (total == 0) return 0;
      if (total > max_sparse) return -1;
      std::memcpy(hbuf, off.data(), k * sizeof(int));
      CHFSI_HIP(hipMemcpyAsync(offsets, hbuf, k * sizeof(int), hipMemcpyHostToDevice, st));
      jacobi_list(g0, k, nr + 1, THR, tau, ratio, offsets, pairs, st);
      CHFSI_HIP(hipMemcpyAsync(hbuf, pairs, 2 * total * sizeof(int), hipMemcpyDeviceToHost, st));
      sync();
      const int* hp = reinterpret_cast<const int*>(hbuf);
      // greedy assignment of each pair to the first round where both of its
      // indices are free
      std::vector<std::vector<int>> rounds;
      std::vector<uint64_t> busy((size_t)k, 0);
      for (int64_t t = 0; t < total; t++) {
        const int p = hp[2 * t], q = hp[2 * t + 1];
        const uint64_t free_mask = ~(busy[p] | busy[q]);
        if (!free_mask) return -1;
        const int r = __builtin_ctzll(free_mask);
        if (r >= max_rounds) return -1;
        if ((int)rounds.size() <= r) rounds.resize(r + 1);
        rounds[r].push_back(p);
        rounds[r].push_back(q);
        busy[p] |= (1ull << r);
        busy[q] |= (1ull << r);
      }
      // device layout per round: pairs (2 np ints), then pair index per row (k ints)
      int* hr = reinterpret_cast<int*>(hbuf);
      size_t pos = 0;
      std::vector<size_t> start(rounds.size());
      for (size_t r = 0; r < rounds.size(); r++) {
        start[r] = pos;
        std::memcpy(hr + pos, rounds[r].data(), rounds[r].size() * sizeof(int));
        pos += rounds[r].size();
        int* po = hr + pos;
        for (int64_t i = 0; i < k; i++) po[i] = -1;
        for (size_t a = 0; a < rounds[r].size() / 2; a++) {
          po[rounds[r][2 * a]] = (int)a;
          po[rounds[r][2 * a + 1]] = (int)a;
        }
        pos += k;
      }
      CHFSI_HIP(hipMemcpyAsync(rounds_d, hr, pos * sizeof(int), hipMemcpyHostToDevice, st));
      fill_i32(flags.i() + 1, 1, 0, st);
      for (size_t r = 0; r < rounds.size(); r++) {
        const int np = (int)(rounds[r].size() / 2);
        const int* pr = rounds_d + start[r];
        jacobi_sparse_round(g0, z0, k, pr, np, pr + 2 * np, jrot.p, nr + 1, tau, flags.i() + 1, st);
      }
      return total;
    };
    for (int sweep = 0; sweep < 100; sweep++) {
      if (refine(g0, sweep > 0 ? z0 : nullptr, k, w, Zo, ldz, tau)) return;
      if (sparse_sweep(REF_ETA) > 0) continue;  // strong couplings only
      const int64_t total = sparse_sweep(0.0);
      if (total == 0) break;
      if (total > 0) continue;
      // dense sweep, block-ordered (two launches per round of blocks)
      fill_i32(flags.i() + 1, 1, 0, st);
      bjv.ensure(block_jacobi_v_bytes(k));
      const int64_t nrounds = block_jacobi_rounds(k);
      for (int64_t r = 0; r < nrounds; r++)
        block_jacobi_round(g0, z0, k, r, nr + 1, tau, bjv.z(), flags.i() + 1, st);
    }
    jacobi_sort(g0, z0, k, w, rank.i(), Zo, ldz, st);
  }

  // Eigen-decomposition of a nearly diagonal Hermitian Gm (k x k, ld k) by
  // iterative refinement of X = I (refine_coeffs).  Zpre (nullable, k x k)
  // holds rotations already applied to the caller's matrix; the result is
  // Zpre X.  Returns false, with w and Zo untouched, when some coupled pair's
  // first correction exceeds ETA (the matrix is not close enough to diagonal
  // for the iteration to converge fast), a later one exceeds GROW, or the
  // corrections do not fall below DONE within MAX_STEPS steps; the caller
  // then continues with Jacobi.  The corrections shrink quadratically
  // (e.g. 0.2, 9e-3, 7e-4, 1e-6, 1e-13), so after a step whose largest
  // correction is below DONE the remaining error is at rounding level.
  static constexpr double REF_ETA = 0.25;
  static constexpr int REF_SPECULATE = 2;  // steps issued before the first read (see refine)
  bool refine_ok_last = false;             // the last first attempt of refine succeeded
  static constexpr int64_t SMALL_REFINE_MIN = 24;
  bool refine(const zc* Gm, const zc* Zpre, int64_t k, double* w, zc* Zo, int64_t ldz, double tau) {
    const double ETA = REF_ETA, GROW = 0.5, DONE = 1e-8;
    const int MAX_STEPS = 10;
    const int64_t kk = k * k;
    zc* X = rf.z();
    zc* Xn = X + kk;
    zc* Wb = Xn + kk;
    zc* Sb = Wb + kk;
    zc* Pb = Sb + kk;
    zc* Eb = Pb + kk;
    double* lam = rfl.d();
    // step 0 puts its largest correction in slot 2; step s >= 1 accumulates
    // in slot s % 2 and clears the other slot for step s + 1 (in stream
    // order; the host reads the slot of the last step of a run of steps)
    auto* corr = static_cast<unsigned long long*>(rfc.p);
    auto read_corr = [&](int step) {
      CHFSI_HIP(hipMemcpyAsync(hbuf, corr + (step == 0 ? 2 : (step & 1)), sizeof(double), hipMemcpyDeviceToHost, st));
      sync();
      double c;
      std::memcpy(&c, hbuf, sizeof(double));
      return c;
    };
    auto run_step = [&](int step) {
      gemm(OP_N, OP_N, k, k, k, 1.0, Gm, k, X, k, Wb, k);
      gemm(OP_C, OP_N, k, k, k, 1.0, X, k, Wb, k, Sb, k);
      gemm(OP_C, OP_N, k, k, k, 1.0, X, k, X, k, Pb, k);
      refine_coeffs(Sb, Pb, k, tau, Eb, nullptr, lam, corr + (step & 1), corr + ((step + 1) & 1), st);
      gemm(OP_N, OP_N, k, k, k, 1.0, X, k, Eb, k, Xn, k, 1.0, X, k);  // X + X E
      std::swap(X, Xn);
    };
    // step 0: X = I, S = Gm, P = I
    CHFSI_HIP(hipMemsetAsync(corr + 2, 0, sizeof(unsigned long long), st));
    refine_coeffs(Gm, nullptr, k, tau, Eb, X, lam, corr + 2, corr + 1, st);
    int step = 1;
    double c;
    // a first attempt after the context's previous one succeeded (the
    // projected matrices of consecutive iterations are alike): the usual
    // first steps run before the first read, which then checks step 0's
    // correction against ETA and the last one against GROW in one wait
    const bool speculate = !Zpre && refine_ok_last;
    if (speculate) {
      for (int i = 0; i < REF_SPECULATE; i++, step++) run_step(step);
      CHFSI_HIP(hipMemcpyAsync(hbuf, corr + 2, sizeof(double), hipMemcpyDeviceToHost, st));
      CHFSI_HIP(hipMemcpyAsync(hbuf + 1, corr + ((step - 1) & 1), sizeof(double), hipMemcpyDeviceToHost, st));
      sync();
      double c0;
      std::memcpy(&c0, hbuf, sizeof(double));
      std::memcpy(&c, hbuf + 1, sizeof(double));
      if (!(c0 <= ETA) || !(c <= GROW)) {
        refine_ok_last = false;
        return false;
      }
    } else {
      c = read_corr(0);
      if (!(c <= ETA)) {
        if (!Zpre) refine_ok_last = false;
        return false;
      }
    }
    // a first attempt records its outcome for the next one
    auto fail = [&]() {
      if (!Zpre) refine_ok_last = false;
      return false;
    };
    while (!(c < DONE)) {
      // the steps that quadratic convergence (c' <= 8 c^2; measured factors
      // 0.2-9) needs to bring the correction below DONE, at most 4, are
      // issued back to back and the correction is read after the last: a
      // step that diverged leaves the last correction above GROW (or NaN)
      int ahead = 0;
      for (double cp = c; ahead < 4 && (ahead == 0 || !(cp < DONE)); ahead++) cp = 8.0 * cp * cp;
      for (int i = 0; i < ahead; i++, step++) {
        if (step > MAX_STEPS) return fail();
        run_step(step);
      }
      c = read_corr(step - 1);
      if (!(c <= GROW)) return fail();
    }
    if (!Zpre) refine_ok_last = true;
    const zc* Zf = X;
    if (Zpre) {
      gemm(OP_N, OP_N, k, k, k, 1.0, Zpre, k, X, k, Wb, k);
      Zf = Wb;
    }
    sort_by_values(lam, Zf, k, w, rank.i(), Zo, ldz, st);
    return true;
  }

  // ------------------------------------------------------------------------
  // Householder QR of F (n x k, ld n, destroyed) into Qo (n x k, ld ldq)
  // ------------------------------------------------------------------------
  void qr(zc* Fp, int64_t ldf, int64_t k, zc* Qo, int64_t ldq) {
    const int64_t npan = cdiv(k, HH_NB);
    for (int64_t p = 0; p < npan; p++) {
      const int64_t j0 = p * HH_NB, j1 = std::min(k, j0 + HH_NB), cnt = j1 - j0;
      HHPanel P{};
      P.F = Fp; P.ldf = ldf; P.n = n; P.j0 = j0; P.j1 = j1;
      P.part = hpart.z(); P.top = htop.z(); P.tau = tau.z();
      hh_panel_setup(P);
      hh_first_partials(P, st);
      for (int64_t j = j0; j < j1; j++) hh_column(P, j, st);
      hh_extract_v(Fp, ldf, n, j0, j1, Vp.z(), n, st);
      const int64_t rows = n - j0;
      gemm(OP_C, OP_N, cnt, cnt, rows, 1.0, Vp.z(), n, Vp.z(), n, gram.z(), cnt);
      zc* Tp = Tall.z() + p * HH_NB * HH_NB;
      hh_build_t(gram.z(), tau.z() + j0, cnt, Tp, st);
      if (j1 < k) {
        const int64_t nc = k - j1;
        zc* C = Fp + j0 + j1 * ldf;
        gemm(OP_C, OP_N, cnt, nc, rows, 1.0, Vp.z(), n, C, ldf, Wt.z(), HH_NB);
        gemm(OP_C, OP_N, cnt, nc, cnt, 1.0, Tp, HH_NB, Wt.z(), HH_NB, W2.z(), HH_NB);
        gemm(OP_N, OP_N, rows, nc, cnt, -1.0, Vp.z(), n, W2.z(), HH_NB, C, ldf, 1.0, C, ldf);
      }
    }
    set_identity(Qo, ldq, n, k, st);
    for (int64_t p = npan - 1; p >= 0; p--) {
      const int64_t j0 = p * HH_NB, j1 = std::min(k, j0 + HH_NB), cnt = j1 - j0;
      const int64_t rows = n - j0, nc = k - j0;
      hh_extract_v(Fp, ldf, n, j0, j1, Vp.z(), n, st);
      zc* C = Qo + j0 + j0 * ldq;
      const zc* Tp = Tall.z() + p * HH_NB * HH_NB;
      gemm(OP_C, OP_N, cnt, nc, rows, 1.0, Vp.z(), n, C, ldq, Wt.z(), HH_NB);
      gemm(OP_N, OP_N, cnt, nc, cnt, 1.0, Tp, HH_NB, Wt.z(), HH_NB, W2.z(), HH_NB);
      gemm(OP_N, OP_N, rows, nc, cnt, -1.0, Vp.z(), n, W2.z(), HH_NB, C, ldq, 1.0, C, ldq);
    }
  }

  // ------------------------------------------------------------------------
  // One CholeskyQR pass: G = Yin^H Yin = Lg Lg^H, Qo = Yin Lg^{-H}.
  // ------------------------------------------------------------------------
  // (The Cholesky reads only the Gram matrix's lower triangle.)  The pass's
  // success lands in info_d (INT_MAX: positive definite) without a wait;
  // Qo is meaningless when it failed.  cond_d (nullable): the ratio of the
  // factor's largest to smallest diagonal entry, a lower bound on cond(Yin).
  void cholqr_pass(const zc* Yin, int64_t ldy, int64_t k, zc* Qo, int64_t ldq, int* info_d, double* cond_d = nullptr) {
    // (lower triangle only: the factorization reads no other part)
    gemm(OP_C, OP_N, k, k, n, 1.0, Yin, ldy, Yin, ldy, G.z(), k, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_OUT_LOWER);
    chol_factor(k, G.z(), k, G2.z(), Z2.z(), Ztmp.z(), k, info_d);
    if (cond_d) diag_ratio(Z2.z(), k, k, cond_d, st);
    gemm(OP_N, OP_C, n, k, k, 1.0, Yin, ldy, Ztmp.z(), k, Qo, ldq, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_TRI_B_UPPER);
  }

  // The passes' outcomes (infos at flags[2], flags[3]) and the first pass's
  // condition estimate with one wait.
  struct CholQROutcome {
    bool first, second;
    double cond;
  };
  CholQROutcome cholqr_outcome() {
    CHFSI_HIP(hipMemcpyAsync(hbuf, flags.i() + 2, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    CHFSI_HIP(hipMemcpyAsync(hbuf + 1, norms.d() + COND_SLOT, sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
    int h[2];
    std::memcpy(h, hbuf, sizeof(h));
    return {h[0] == INT_MAX, h[1] == INT_MAX, hbuf[1]};
  }

  // CholeskyQR2 leaves Q orthonormal to working precision when the first
  // pass's orthogonality error (about eps cond(F)^2) is small; its Cholesky
  // succeeds up to cond(F) near 1e8.  Between a condition estimate of
  // COND_GRAY and that breakdown the second pass may leave a visible loss,
  // so a third pass runs there (its Gram matrix is then close to I).
  static constexpr double COND_GRAY = 1e6;
  static constexpr int COND_SLOT = 6;  // norms slot of the condition estimate

  // Orthonormal basis of span(F) (F: n x k, ld n, destroyed) into Qo.
  // CholeskyQR2 (a third pass above the gray-zone estimate); if a Gram
  // matrix is not positive definite the block is too ill-conditioned for
  // it and Householder QR takes over on the best basis at hand.  Returns
  // true when Householder was used.
  bool orthonormalize(zc* Fp, int64_t k, zc* Qo, int64_t ldq) {
    return orthonormalize_active(nullptr, Fp, 0, k, Qo, ldq);
  }

  // Orthonormal basis of [Y_lock | F(:, cl:k)] with the locked columns
  // Y_lock = Yl(:, :cl) (orthonormal) kept: two passes of block classical
  // Gram-Schmidt of the active columns against Y_lock followed by CholeskyQR
  // of the remainder -- CholeskyQR2 of the whole block with the locked
  // block's Gram matrix and Cholesky factor (the identity) taken as known,
  // so the factorization is k_a x k_a instead of k x k.  Result in
  // Qo(:, cl:k).  When a Gram matrix is not positive definite, Householder
  // QR of the whole block (F(:, :cl) gets Y_lock) writes all of Qo; returns
  // true then.
  bool orthonormalize_active(const zc* Yl, zc* Fp, int64_t cl, int64_t k, zc* Qo, int64_t ldq) {
    const int64_t ka = k - cl;
    if (opts.qr_mode == 0) {
      zc* Fa = Fp + cl * n;
      zc* mid = Wk.z();
      zc* B = Z2.z();  // cl x ka coefficients (Z2 is free between the passes' factorizations)
      auto project = [&](zc* X, int64_t ldx) {
        if (cl == 0) return;
        gemm(OP_C, OP_N, cl, ka, n, 1.0, Yl, n, X, ldx, B, cl);
        gemm(OP_N, OP_N, n, ka, cl, -1.0, Yl, n, B, cl, X, ldx, 1.0, X, ldx);  // X -= Y_lock B
      };
      zc* Qa = Qo + cl * ldq;
      project(Fa, n);
      cholqr_pass(Fa, n, ka, mid, n, flags.i() + 2, norms.d() + COND_SLOT);
      project(mid, n);
      cholqr_pass(mid, n, ka, Qa, ldq, flags.i() + 3);
      const CholQROutcome ok = cholqr_outcome();
      if (ok.first && ok.second) {
        if (!(ok.cond > COND_GRAY)) return false;
        // gray zone: one more pass on the second pass's result
        project(Qa, ldq);
        cholqr_pass(Qa, ldq, ka, mid, n, flags.i() + 2);
        fill_i32(flags.i() + 3, 1, INT_MAX, st);
        const CholQROutcome ok3 = cholqr_outcome();
        if (ok3.first) {
          copy2d(mid, n, Qa, ldq, n, ka, st);
          return false;
        }
        copy2d(Qa, ldq, Fa, n, n, ka, st);  // Householder from the second pass's basis
      } else if (ok.first) {
        copy2d(mid, n, Fa, n, n, ka, st);  // from the first pass's, far better conditioned than F
      }
    }
    if (cl > 0) copy2d(Yl, n, Fp, n, n, cl, st);
    qr(Fp, n, k, Qo, ldq);
    return true;
  }

  // ------------------------------------------------------------------------
  // Chebyshev filter on Y (n x ka); Yb same shape as work.  Returns the
  // buffer holding the result (Y or Yb).
  // ------------------------------------------------------------------------
  // AY0 (optional, FP64): A Y_0 already at hand (the Rayleigh-Ritz step's
  // W Z for the Ritz vectors in Y_0); the first step then needs no product.
  zc* filter(const zc* Ap, int64_t lda, zc* Yp, int64_t ldy, zc* Ybp, int64_t ldyb, int64_t ka, int m, double a, double b,
             double a0, const zc* AY0 = nullptr, int64_t lday = 0) {
    return static_cast<zc*>(filter_any(PREC_F64, Ap, lda, Yp, ldy, Ybp, ldyb, ka, m, a, b, a0, AY0, lday));
  }

  // The filter in either precision: element type zc (FP64) or cc (FP32).
  void* filter_any(int prec, const void* Ap, int64_t lda, void* Yp, int64_t ldy, void* Ybp, int64_t ldyb, int64_t ka, int m,
                   double a, double b, double a0, const zc* AY0 = nullptr, int64_t lday = 0) {
    const bool prof = opts.profile != 0;
    // profile mode: one event pair around the call's consecutive degree
    // steps (a pair per step would put a timed marker between every two
    // launches, which on this runtime costs the stream a few microseconds
    // each); the per-launch figure then includes the short gaps between
    // back-to-back launches
    std::vector<EventPair>& ev = fev[prec];
    if (prof && ev.empty()) {
      EventPair ep;
      CHFSI_HIP(hipEventCreate(&ep.a));
      CHFSI_HIP(hipEventCreate(&ep.b));
      ev.push_back(ep);
    }
    auto step = [&](const void* cur, int64_t ldc, void* out, int64_t ldo, double al, double be, double ga,
                    const void* prev, int64_t ldp) {
      GemmOp g;
      g.prec = prec;
      g.M = n; g.N = ka; g.K = n;
      g.A = Ap; g.lda = lda; g.B = cur; g.ldb = ldc; g.C = out; g.ldc = ldo;
      g.X = cur; g.ldx = ldc; g.Z = prev; g.ldz = ldp;
      g.alpha = al; g.beta = be; g.gamma = ga;
      g.filter_step = true;
      g.cfg = opts.filter_tile;
      g.splitk = opts.filter_splitk;
      zgemm(g, gw(), st);
    };
    const std::vector<ChebStep> cs = cheb_schedule(m, a, b, a0);
    // Y_1 = (sigma1/e)(A - cI) Y_0
    const bool reuse = AY0 && prec == PREC_F64;
    if (reuse)
      lincomb2d(cs[0].alpha, AY0, lday, cs[0].beta, static_cast<const zc*>(Yp), ldy, static_cast<zc*>(Ybp), ldyb, n, ka, st);
    if (prof) CHFSI_HIP(hipEventRecord(ev[0].a, st));
    if (!reuse) step(Yp, ldy, Ybp, ldyb, cs[0].alpha, cs[0].beta, 0.0, nullptr, 0);
    void *cur = Ybp, *prev = Yp;
    int64_t ldc = ldyb, ldp = ldy;
    for (int i = 1; i < m; i++) {
      // Y_{i+1} = alpha (A - cI)-scaled product - sigma sigma' Y_{i-1}, over Y_{i-1}
      step(cur, ldc, prev, ldp, cs[i].alpha, cs[i].beta, cs[i].gamma, prev, ldp);
      std::swap(cur, prev);
      std::swap(ldc, ldp);
    }
    if (prof) CHFSI_HIP(hipEventRecord(ev[0].b, st));
    const int products = reuse ? m - 1 : m;
    filt_launches[prec] += products;
    filt_flops[prec] += 8.0 * (double)n * (double)n * (double)ka * (double)products;
    if (prof) filt_pending[prec] = true;
    return cur;
  }

  // The filter of Y_0 (n x ka, FP64 Ritz vectors of A with Ritz values mu,
  // AY0 = A Y_0 in FP64) with its matrix products in complex FP32 (or, with
  // half, FP16 operands and FP32 accumulation), result F (FP64).  The
  // recurrence of eq. (2) is linear, so its iterates split as
  // Y_i = Y_0 diag(t_i(mu)) + D_i, with t_i the same recurrence on the
  // scalars mu_j (FP64, on the host) and D_i the recurrence on the Ritz
  // residual R = A Y_0 - Y_0 diag(mu):
  //   D_0 = 0, D_1 = alpha_0 R,
  //   D_{i+1} = alpha_i A D_i + beta_i D_i + gamma_i D_{i-1} + alpha_i t_i(mu) R.
  // Only D runs in the lower precision (A rounded to it in A32 / A16, each
  // column of D scaled by a power of two to unit size); its rounding errors
  // are relative to |D|, which shrinks with the residual, so the filtered
  // block keeps FP64 accuracy where Y_0 has converged (the plain FP32
  // filter's errors are relative to |Y_i| and stop convergence near
  // 1e-7 ||A||).  mu_d (device) and mu_h (host) hold the same ka values.
  void filter_ritz(const zc* Y0, int64_t ldy, const zc* AY0, int64_t lday, const double* mu_d, const double* mu_h,
                   int64_t ka, int m, double a, double b, double a0, zc* F, int64_t ldf, bool half) {
    if (ka < 1) return;
    const bool prof = opts.profile != 0;
    std::vector<EventPair>& ev = fev[PREC_F32];
    if (prof && ev.empty()) {
      EventPair ep;
      CHFSI_HIP(hipEventCreate(&ep.a));
      CHFSI_HIP(hipEventCreate(&ep.b));
      ev.push_back(ep);
    }
    const std::vector<ChebStep> cs = cheb_schedule(m, a, b, a0);
    cc* cur = (cc*)Y32b.p;
    cc* prev = (cc*)Y32.p;
    ritz_prepare(Y0, ldy, AY0, lday, mu_d, mu_h, ka, cs, cur);
    // FP16 steps: each iterate also as FP16 planes (written by the step
    // that forms it, read as the next step's operand); rows n .. ld16 - 1
    // stay zero
    const int64_t ld16 = f16_plane_ld(n), pl16 = ka * ld16;
    _Float16 *h_cur = nullptr, *h_prev = nullptr;
    if (half && m > 1) {
      const size_t bytes = (size_t)4 * pl16 * sizeof(_Float16);
      D16.ensure(bytes);
      CHFSI_HIP(hipMemsetAsync(D16.p, 0, bytes, st));
      h_cur = (_Float16*)D16.p;
      h_prev = h_cur + 2 * pl16;
      to_f16_cols(cur, n, n, ka, h_cur, ld16, pl16, st);
    }
    if (prof) CHFSI_HIP(hipEventRecord(ev[0].a, st));
    for (int i = 1; i < m; i++) {
      GemmOp g;
      g.prec = PREC_F32;
      g.M = n; g.N = ka; g.K = n;
      g.A = half ? A16.p : A32.p;
      g.lda = half ? f16_plane_ld(n) : n;
      g.B = cur; g.ldb = n; g.C = prev; g.ldc = n;
      g.X = cur; g.ldx = n;
      g.Z = i == 1 ? nullptr : prev;  // D_0 = 0
      g.ldz = n;
      g.alpha = cs[i].alpha; g.beta = cs[i].beta; g.gamma = cs[i].gamma;
      g.R = R32.p; g.ldr = n; g.rs = ctab.d() + (size_t)i * ka;
      g.filter_step = true;
      if (half) {
        g.cfg = opts.filter_tile;
        g.splitk = opts.filter_splitk;
        g.B16 = h_cur;
        g.C16 = i + 1 < m ? h_prev : nullptr;  // the last iterate feeds no product
        g.ld16 = ld16;
        g.pl16 = pl16;
        zgemm_f16_step(g, gw(), st);
        std::swap(h_cur, h_prev);
      } else {
        g.cfg = opts.filter_tile;
        g.splitk = opts.filter_splitk;
        zgemm(g, gw(), st);
      }
      std::swap(cur, prev);
    }
    if (prof) CHFSI_HIP(hipEventRecord(ev[0].b, st));
    ritz_finish(Y0, ldy, cur, m, ka, F, ldf);
    filt_launches[PREC_F32] += m - 1;
    filt_flops[PREC_F32] += 8.0 * (double)n * (double)n * (double)ka * (double)(m - 1);
    if (prof && m > 1) filt_pending[PREC_F32] = true;
  }

  // The parts of the Ritz-residual filter around its products: the scalar
  // recurrence's table on the device (rows 1..m-1: the forcing scale
  // alpha_i t_i(mu_j) of step i; row m: t_m(mu_j); row m + 1: the columns'
  // scales, written by the device), R into R32 and D_1 into D1 (n x ka,
  // FP32, both divided by the column scales); then
  // F = Y_0 diag(t_m) + D_m diag(scale).
  void ritz_prepare(const zc* Y0, int64_t ldy, const zc* AY0, int64_t lday, const double* mu_d, const double* mu_h,
                    int64_t ka, const std::vector<ChebStep>& cs, cc* D1) {
    const int m = (int)cs.size();
    const size_t tab_elems = (size_t)(m + 1) * ka;
    ensure_htab(tab_elems);
    ctab.ensure((tab_elems + ka) * sizeof(double));
    double* tab = htab;
    for (int64_t j = 0; j < ka; j++) {
      const double mj = mu_h[j];
      double tp = 1.0, t = fma(cs[0].alpha, mj, cs[0].beta);
      for (int i = 1; i < m; i++) {
        tab[(size_t)i * ka + j] = cs[i].alpha * t;
        const double tn = cs[i].alpha * mj * t + cs[i].beta * t + cs[i].gamma * tp;
        tp = t;
        t = tn;
      }
      tab[(size_t)m * ka + j] = t;
    }
    CHFSI_HIP(hipMemcpyAsync(ctab.p, tab, tab_elems * sizeof(double), hipMemcpyHostToDevice, st));
    ritz_forcing(Y0, ldy, AY0, lday, mu_d, cs[0].alpha, (cc*)R32.p, n, D1, n, ctab.d() + tab_elems, n, ka, st);
  }

  void ritz_finish(const zc* Y0, int64_t ldy, const cc* Dm, int m, int64_t ka, zc* F, int64_t ldf) {
    const size_t tab_elems = (size_t)(m + 1) * ka;
    ritz_combine(Y0, ldy, ctab.d() + (size_t)m * ka, ctab.d() + tab_elems, Dm, n, F, ldf, n, ka, st);
  }

  // Add the event time of the filter run since the last call in each
  // precision (the stream must have passed it).
  void collect_filter_events() {
    for (int p = 0; p < 2; p++) {
      if (!filt_pending[p] || fev[p].empty()) continue;
      float ms = 0.f;
      CHFSI_HIP(hipEventElapsedTime(&ms, fev[p][0].a, fev[p][0].b));
      filt_kernel_s[p] += ms * 1e-3;
      filt_pending[p] = false;
    }
  }

  // ------------------------------------------------------------------------
  // Rayleigh-Ritz on Qa (n x ka, orthonormal) -> Yo = Qa Z, mu (device),
  // WZo = A Yo (through W Z).
  // ------------------------------------------------------------------------
  void rayleigh_ritz(const zc* Ap, int64_t lda, const zc* Qa, int64_t ldq, int64_t ka, zc* Yo, int64_t ldyo, double* mu_d,
                     zc* Wbuf, zc* WZo, double tau = 0.0) {
    gemm(OP_N, OP_N, n, ka, n, 1.0, Ap, lda, Qa, ldq, Wbuf, n);
    // the lower triangle of Q^H W, mirrored: an exactly Hermitian G
    gemm(OP_C, OP_N, ka, ka, n, 1.0, Qa, ldq, Wbuf, n, G.z(), ka, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_OUT_LOWER);
    hermitian_from_lower(G.z(), ka, ka, st);
    eigh(G.z(), ka, ka, mu_d, Z.z(), ka, tau);
    gemm(OP_N, OP_N, n, ka, ka, 1.0, Qa, ldq, Z.z(), ka, Yo, ldyo);
    if (WZo) gemm(OP_N, OP_N, n, ka, ka, 1.0, Wbuf, n, Z.z(), ka, WZo, n);
  }

  // rho_j = || L (WZ_j - mu_j y_j) ||
  void residual_norms(const zc* Lp, int64_t ldl, const zc* WZ, const zc* Yp, int64_t ldy, int64_t ka, const double* mu_d,
                      zc* Rbuf, zc* LRbuf, double* rho_d) {
    residual_block(WZ, n, Yp, ldy, mu_d, Rbuf, n, n, ka, st);
    gemm(OP_N, OP_N, n, ka, n, 1.0, Lp, ldl, Rbuf, n, LRbuf, n, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_TRI_A_LOWER);
    column_norms(LRbuf, n, n, ka, rho_d, st);
  }

  // ------------------------------------------------------------------------
  // Lanczos (full re-orthogonalization): out = {theta_min, theta_max, b}
  // ------------------------------------------------------------------------
  void lanczos(const zc* Ap, int64_t lda, int steps, uint64_t seed, uint32_t sid, double out[3]) {
    ensure_small();
    steps = (int)std::min<int64_t>(std::min<int64_t>(steps, n), JACOBI_LDS_MAX);
    if (steps < 1) throw Error(ST_EINVAL, "lanczos: steps < 1");
    zc* V = LV.z();
    zc* w = Lw.z();
    zc* h = Lh.z();
    double* alpha = Lab.d();
    double* beta = Lab.d() + (steps + 2);
    random_block(seed, sid, n, 1, 0, w, n, st);
    normalize(w, n, V, beta, st);  // beta[0] = ||v0|| (unused afterwards)
    for (int j = 0; j < steps; j++) {
      zgemv(Ap, lda, n, V + (int64_t)j * n, w, mvpart.z(), st);
      multi_dot(V + (int64_t)j * n, n, n, 1, w, h, st);
      lanczos_three_term(w, V, n, n, j, alpha, beta, h, st);
      for (int pass = 0; pass < 2; pass++) {
        multi_dot(V, n, n, j + 1, w, h, st);
        sub_combination(V, n, n, j + 1, h, w, st);
      }
      normalize(w, n, V + (int64_t)(j + 1) * n, beta + j + 1, st);
    }
    std::vector<double> ab(2 * (steps + 2));
    CHFSI_HIP(hipMemcpyAsync(hbuf, Lab.p, ab.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
    std::memcpy(ab.data(), hbuf, ab.size() * sizeof(double));
    const double* al = ab.data();
    const double* be = ab.data() + (steps + 2);
    int used = steps;
    for (int j = 0; j + 1 < steps; j++)
      if (!(be[j + 1] > 0.0)) {
        used = j + 1;
        break;
      }
    const double fnorm = be[used];
    std::vector<zc> T((size_t)used * used, zmk(0.0, 0.0));
    for (int i = 0; i < used; i++) {
      T[i + (size_t)i * used] = zmk(al[i], 0.0);
      if (i + 1 < used) {
        T[(i + 1) + (size_t)i * used] = zmk(be[i + 1], 0.0);
        T[i + (size_t)(i + 1) * used] = zmk(be[i + 1], 0.0);
      }
    }
    std::memcpy(hbuf, T.data(), T.size() * sizeof(zc));
    CHFSI_HIP(hipMemcpyAsync(Tsm.p, hbuf, T.size() * sizeof(zc), hipMemcpyHostToDevice, st));
    jacobi_small(Tsm.z(), used, used, Tw.d(), Tz.z(), used, Tz2.z(), nullptr, st);
    std::vector<double> th(used);
    CHFSI_HIP(hipMemcpyAsync(hbuf + 2 * JACOBI_LDS_MAX * JACOBI_LDS_MAX, Tw.p, used * sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
    std::memcpy(th.data(), hbuf + 2 * JACOBI_LDS_MAX * JACOBI_LDS_MAX, used * sizeof(double));
    out[0] = th[0];
    out[1] = th[used - 1];
    out[2] = th[used - 1] + fnorm;
  }
};

namespace {

template <class F>
chfsi_status guarded(chfsi_ctx c, F&& f) {
  if (!c) return CHFSI_EINVAL;
  try {
    c->err.clear();
    f();
    return CHFSI_OK;
  } catch (const Error& e) {
    c->err = e.what();
    (void)hipGetLastError();
    return (chfsi_status)e.code;
  } catch (const std::exception& e) {
    c->err = e.what();
    return CHFSI_EHIP;
  } catch (...) {
    c->err = "unknown error";
    return CHFSI_EHIP;
  }
}

void check_ld(int64_t ld, int64_t rows, const char* name) {
  if (ld < rows || ld < 1) throw Error(ST_EINVAL, std::string("leading dimension ") + name + " smaller than the rows");
}

void check_ptr(const void* p, const char* name) {
  if (!p) throw Error(ST_EINVAL, std::string("null pointer: ") + name);
}

// Algorithm 1 in phases, so that a batch of problems can run its filters in
// shared launches: solve_begin (reduction, Lanczos, start block, bounds),
// then per outer iteration solve_filter (the Chebyshev filter of the active
// columns into F) and solve_post (QR, Rayleigh-Ritz, residuals, locking),
// then solve_finish (outputs and warm state).
struct SolveState {
  const zc* H = nullptr;
  int64_t ldh = 0;
  const zc* S = nullptr;
  int64_t lds = 0;
  int64_t nev = 0, nex = 0, k = 0;
  const zc* Vw = nullptr;
  int64_t ldv = 0, kw = 0;
  double tol = 0;
  double* evals = nullptr;
  zc* X = nullptr;
  int64_t ldx = 0;
  const double* bounds_in = nullptr;

  chfsi_info inf{};
  std::chrono::steady_clock::time_point t_start;
  double a0 = 0, a = 0, b = 0, hs = 0;
  int64_t cl = 0;
  int it = 0;
  bool converged = false, done = false, mixed = false;
  bool ritz = false;    // precision 2 or 3: the filter on the Ritz residual
  bool ritz16 = false;  // precision 3: its products with FP16 operands
  double mixed_switch = 0.0;  // relative residual below which a column's filter is FP64
  std::vector<double> lam, rho_lock;
  std::vector<hipEvent_t> ev;
  // mixed precision: this iteration's leading active columns filtered in
  // FP64 (the rest in FP32), the columns below fp64_upto that stay FP64,
  // the last residual of every column, and the first active column's
  // previous residual for the stall test
  int64_t split = 0, fp64_upto = 0;
  // first column whose A y is in Wz (the last Rayleigh-Ritz step's W Z), or -1
  int64_t wz_first = -1;
  std::vector<double> rho_last;
  int64_t prev_first = -1;
  double prev_first_rho = INFINITY;
  bool prev_first32 = false;

  ~SolveState() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// Mixed precision, per column: the FP64 filter takes the leading active
// columns whose generalized residuals have all reached the switch (MIXED_SWITCH
// unless the options set another) times h_H
// (an order above where FP32 rounding in the filter holds them); the
// columns after the first one still above it are filtered in complex FP32.
// The FP64 range only grows (a column stays FP64 until it locks), and the
// first active column also turns FP64 if an FP32 iteration fails to halve
// its residual.  QR, Rayleigh-Ritz, residuals and locking stay FP64, so
// accepted pairs meet the same tolerance.
constexpr double MIXED_SWITCH = 1e-6;
constexpr int64_t MIXED_MIN_COLS = 64;
// Lockable columns whose residuals an FP64 iteration forms first.
constexpr int64_t RESID_FIRST = 64;

double secs_since(std::chrono::steady_clock::time_point a) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
}

void solve_begin(chfsi_ctx c, SolveState& s) {
  const int64_t n = c->n;
  s.k = s.nev + s.nex;
  // the refinement's speculation starts afresh, so that a solve's steps (and
  // bits) do not depend on what the context solved before
  c->refine_ok_last = false;
  const int64_t k = s.k;
  if (!block_sizes_ok(n, s.nev, s.nex)) throw Error(ST_EINVAL, BLOCK_SIZES_RULE);
  if (!(s.tol > 0.0)) throw Error(ST_EINVAL, "tol must be positive");
  if (s.kw < 0 || s.kw > k) throw Error(ST_EINVAL, "kw out of range");
  check_ptr(s.H, "H");
  check_ld(s.ldh, n, "ldh");
  if (s.S) check_ld(s.lds, n, "lds");
  if (s.Vw && s.kw > 0) check_ld(s.ldv, n, "ldv");
  if (s.X) check_ld(s.ldx, n, "ldx");
  check_ptr(s.evals, "evals");
  const chfsi_opts& o = c->opts;
  hipStream_t st = c->st;
  chfsi_info& inf = s.inf;
  s.t_start = std::chrono::steady_clock::now();
  c->reset_filter_stats();

  c->ensure_nn();
  c->ensure_small();
  // start block: explicit warm vectors, else the block (and filter bounds)
  // kept from the context's previous solve when its width matches, else a
  // seeded random block
  const bool explicit_warm = s.Vw != nullptr && s.kw > 0;
  const bool use_state = !explicit_warm && c->warm_valid && c->have_factors && c->warm_k == k && c->Y.p;
  c->ensure_k(k);

  auto t0 = std::chrono::steady_clock::now();
  roctxRangePushA("chfsi.reduce");
  // (a kept block meant for a changed S is carried to the new factor here)
  try {
    c->reduce(s.H, s.ldh, s.S, s.lds, use_state);
  } catch (...) {
    roctxRangePop();
    throw;
  }
  s.mixed = o.precision == 1;
  s.ritz = o.precision >= 2;
  s.ritz16 = o.precision == 3;
  s.mixed_switch = o.mixed_switch_digits > 0 ? std::pow(10.0, -o.mixed_switch_digits) : MIXED_SWITCH;
  if (s.mixed || s.ritz) {
    c->A32.ensure((size_t)n * n * sizeof(cc));
    c->Y32.ensure((size_t)n * k * sizeof(cc));
    c->Y32b.ensure((size_t)n * k * sizeof(cc));
    if (s.ritz) c->R32.ensure((size_t)n * k * sizeof(cc));
    to_f32(c->A.z(), n, (cc*)c->A32.p, n, n, n, st);
    if (s.ritz16) {
      c->A16.ensure((size_t)2 * n * f16_plane_ld(n) * sizeof(_Float16));
      to_f16_planes(c->A.z(), n, n, c->A16.p, st);
    }
  }
  c->sync();
  roctxRangePop();
  inf.t_reduce = secs_since(t0);

  t0 = std::chrono::steady_clock::now();
  double lz[3];
  {
    Range r_lanczos("chfsi.lanczos");
    c->lanczos(c->A.z(), n, o.lanczos_steps, o.seed, 1u, lz);
    inf.theta_min = lz[0];
    inf.b_upper = lz[2];
    c->lanczos(s.H, s.ldh, o.lanczos_steps, o.seed, 2u, lz);
    inf.h_H = std::max(std::fabs(lz[0]), std::fabs(lz[1]));
  }
  inf.t_lanczos = secs_since(t0);
  Range r_start("chfsi.start_block");

  zc* Y = c->Y.z();
  zc* F = c->F.z();
  zc* Qb = c->Qb.z();
  // start block
  bool warm = false;
  bool start_ritz = false;  // Y holds Ritz vectors, their values in mu, A Y in Wz
  // the kept block survived the reduction (it is in the current standard form)
  const bool kept = use_state && c->warm_valid;
  if (explicit_warm) {
    c->gemm(OP_C, OP_N, n, s.kw, n, 1.0, c->L.z(), n, s.Vw, s.ldv, Y, n, 0.0, nullptr, 0, 0.0, nullptr, 0,
            GEMM_TRI_A_UPPER);
    if (s.kw < k) random_block(o.seed, 3u, n, k - s.kw, s.kw, Y + s.kw * n, n, st);
    warm = true;
  } else if (kept) {
    warm = true;
  } else {
    random_block(o.seed, 3u, n, k, 0, Y, n, st);
  }
  copy2d(Y, n, F, n, n, k, st);
  inf.qr_householder += c->orthonormalize(F, k, Qb, n) ? 1 : 0;
  s.b = inf.b_upper;
  // filter bounds: the caller's; else, for the kept block, the ones kept
  // with it; else (cold start, or explicit vectors without bounds) from one
  // Rayleigh-Ritz step of the start block
  if (warm && s.bounds_in) {
    copy2d(Qb, n, Y, n, n, k, st);
    s.a0 = s.bounds_in[0];
    s.a = s.bounds_in[1];
  } else if (kept) {
    copy2d(Qb, n, Y, n, n, k, st);
    s.a0 = c->warm_a0;
    s.a = c->warm_a;
  } else {
    // the filter on the Ritz residual takes this step's Ritz vectors, values
    // and A Y (W Z) for its first iteration too
    c->rayleigh_ritz(c->A.z(), n, Qb, n, k, Y, n, c->mu.d(), c->Wk.z(), s.ritz ? c->Wz.z() : nullptr);
    double* hb = c->hbuf;
    CHFSI_HIP(hipMemcpyAsync(hb, c->mu.d(), k * sizeof(double), hipMemcpyDeviceToHost, st));
    c->sync();
    s.a0 = std::min(inf.theta_min, hb[0]);
    s.a = hb[k - 1];
    start_ritz = s.ritz;
  }
  inf.warm_start = warm ? 1 : 0;
  c->warm_valid = false;  // the block is being rewritten
  s.lam.assign(k, NAN);
  if (start_ritz) {
    std::copy(c->hbuf, c->hbuf + k, s.lam.begin());
    s.wz_first = 0;
  }
  s.rho_lock.assign(k, 0.0);
  s.rho_last.assign(k, INFINITY);
  s.cl = 0;
  s.it = 0;
  s.hs = s.tol * inf.h_H;
  s.ev.resize(5);
  for (auto& e : s.ev) CHFSI_HIP(hipEventCreate(&e));
}

// Host side of an outer iteration's start: count it and fix the split of
// the active columns between the FP64 and FP32 filters.
void solve_filter_begin(SolveState& s) {
  s.it++;
  const int64_t ka = s.k - s.cl;
  // The damped interval [a, b] must not be empty: when the Lanczos bound is
  // exact (n at most the Lanczos steps) and the block spans the whole space,
  // b equals the largest Ritz value a and the scaled recurrence would divide
  // zero by zero.  Raising b by a relative 1e-8 changes nothing elsewhere.
  s.b = std::max(s.b, s.a + 1e-8 * std::max(std::max(std::fabs(s.a), std::fabs(s.b)),
                                             std::max(s.inf.h_H, 1e-300)));
  if (s.ritz) {
    s.split = 0;  // every active column in the lower precision
    return;
  }
  if (!s.mixed) {
    s.split = ka;
    return;
  }
  int64_t j = std::max(s.cl, s.fp64_upto);
  while (j < s.k && s.rho_last[j] <= s.mixed_switch * s.inf.h_H) j++;
  s.fp64_upto = j;
  s.split = std::min(ka, std::max<int64_t>(0, s.fp64_upto - s.cl));
  // a narrow FP32 part does not pay for its own launches and conversions
  // beside an FP64 one (measured: a warm n = 4000 sequence ran slower in
  // mixed precision than in FP64): filter everything in FP64 then
  if (s.split > 0 && ka - s.split < std::max<int64_t>(MIXED_MIN_COLS, ka / 8)) s.split = ka;
}

// The filter of the active columns, result into F(:, cl:k).
void solve_filter(chfsi_ctx c, SolveState& s) {
  const int64_t n = c->n, ka = s.k - s.cl;
  hipStream_t st = c->st;
  solve_filter_begin(s);
  Range r_filter("chfsi.filter");
  CHFSI_HIP(hipEventRecord(s.ev[0], st));
  zc* Y = c->Y.z();
  zc* F = c->F.z();
  const int64_t p = s.split, c32 = s.cl + p;
  // A Y_0 of the active columns is the last Rayleigh-Ritz step's W Z (and
  // their Ritz values are in mu from the same offset)
  const bool have_wz = s.wz_first >= 0 && s.cl >= s.wz_first;
  const zc* ay0 = have_wz ? c->Wz.z() + (s.cl - s.wz_first) * n : nullptr;
  if (p > 0) {
    zc* res = c->filter(c->A.z(), n, Y + s.cl * n, n, c->Yb.z() + s.cl * n, n, p, c->opts.degree, s.a, s.b, s.a0, ay0, n);
    copy2d(res, n, F + s.cl * n, n, n, p, st);
  }
  if (p < ka && s.ritz && have_wz) {
    // the active columns are Ritz vectors: the filter on their residual
    c->filter_ritz(Y + s.cl * n, n, ay0, n, c->mu.d() + (s.cl - s.wz_first), s.lam.data() + s.cl, ka,
                   c->opts.degree, s.a, s.b, s.a0, F + s.cl * n, n, s.ritz16);
    s.inf.iterations_fp32++;
  } else if (p < ka) {
    cc* y32 = (cc*)c->Y32.p;
    cc* y32b = (cc*)c->Y32b.p;
    to_f32(Y + c32 * n, n, y32, n, n, ka - p, st);
    void* r32 = c->filter_any(PREC_F32, c->A32.p, n, y32, n, y32b, n, ka - p, c->opts.degree, s.a, s.b, s.a0);
    to_f64((const cc*)r32, n, F + c32 * n, n, n, ka - p, st);
    s.inf.iterations_fp32++;
  }
  CHFSI_HIP(hipEventRecord(s.ev[1], st));
}

// QR, Rayleigh-Ritz, residuals and locking after the filter.
void solve_post(chfsi_ctx c, SolveState& s) {
  const int64_t n = c->n, k = s.k, ka = k - s.cl, cl = s.cl;
  hipStream_t st = c->st;
  chfsi_info& inf = s.inf;
  zc* Y = c->Y.z();
  zc* F = c->F.z();
  zc* Qb = c->Qb.z();
  double* mu_d = c->mu.d();
  double* rho_d = c->rho.d();
  {
    Range r_qr("chfsi.qr");
    inf.qr_householder += c->orthonormalize_active(Y, F, cl, k, Qb, n) ? 1 : 0;
  }
  CHFSI_HIP(hipEventRecord(s.ev[2], st));
  {
    Range r_rr("chfsi.rayleigh_ritz");
    c->rayleigh_ritz(c->A.z(), n, Qb + cl * n, n, ka, Y + cl * n, n, mu_d, c->Wk.z(), c->Wz.z(), 1e-3 * s.hs);
  }
  CHFSI_HIP(hipEventRecord(s.ev[3], st));
  Range r_lock("chfsi.residuals_lock");
  // residuals of the columns that can lock (at most nev - cl of them: the
  // extra columns never do); mixed precision reads every active column's
  // residual for its precision rules
  const int64_t kr = s.mixed ? ka : std::min(ka, s.nev - cl);
  // FP64: the residuals of the first RESID_FIRST of those columns, and of
  // the rest only when all of these lock (the lock takes a contiguous
  // prefix, so no column after the first one above the tolerance can lock
  // this iteration; until the first columns converge, most of the
  // triangular product L R is skipped)
  const int64_t kr1 = s.mixed ? kr : std::min(kr, RESID_FIRST);
  c->residual_norms(c->L.z(), n, c->Wz.z(), Y + cl * n, n, kr1, mu_d, c->Wk.z(), F, rho_d);
  s.wz_first = cl;  // Wz = A Y(:, cl:k) until the next Rayleigh-Ritz step
  double* hb = c->hbuf;
  CHFSI_HIP(hipMemcpyAsync(hb, mu_d, ka * sizeof(double), hipMemcpyDeviceToHost, st));
  CHFSI_HIP(hipMemcpyAsync(hb + ka, rho_d, kr1 * sizeof(double), hipMemcpyDeviceToHost, st));
  CHFSI_HIP(hipEventRecord(s.ev[4], st));
  c->sync();
  float ms[4];
  for (int i = 0; i < 4; i++) CHFSI_HIP(hipEventElapsedTime(&ms[i], s.ev[i], s.ev[i + 1]));
  inf.t_filter += ms[0] * 1e-3;
  inf.t_qr += ms[1] * 1e-3;
  inf.t_rr += ms[2] * 1e-3;
  inf.t_resid += ms[3] * 1e-3;
  c->collect_filter_events();
  const double* mu = hb;
  double* rho = hb + ka;
  for (int64_t j = 0; j < ka; j++)
    if (!std::isfinite(mu[j]) || (j < kr1 && !std::isfinite(rho[j])))
      throw Error(ST_ENAN, "non-finite Ritz value or residual at iteration " + std::to_string(s.it));
  for (int64_t j = kr1; j < ka; j++) rho[j] = INFINITY;  // not formed
  int64_t nl = 0;
  while (cl + nl < s.nev && nl < ka && rho[nl] <= s.hs) nl++;
  if (nl == kr1 && kr1 < kr) {
    // every column of the first part locks: the residuals of the rest
    const auto t1 = std::chrono::steady_clock::now();
    c->residual_norms(c->L.z(), n, c->Wz.z() + kr1 * n, Y + (cl + kr1) * n, n, kr - kr1, mu_d + kr1, c->Wk.z(), F,
                      rho_d + kr1);
    CHFSI_HIP(hipMemcpyAsync(rho + kr1, rho_d + kr1, (kr - kr1) * sizeof(double), hipMemcpyDeviceToHost, st));
    c->sync();
    inf.t_resid += secs_since(t1);
    for (int64_t j = kr1; j < kr; j++)
      if (!std::isfinite(rho[j]))
        throw Error(ST_ENAN, "non-finite residual at iteration " + std::to_string(s.it));
    while (cl + nl < s.nev && nl < ka && rho[nl] <= s.hs) nl++;
  }
  for (int64_t j = 0; j < nl; j++) {
    s.lam[cl + j] = mu[j];
    s.rho_lock[cl + j] = rho[j];
  }
  for (int64_t j = nl; j < ka; j++) {
    s.lam[cl + j] = mu[j];
    s.rho_lock[cl + j] = rho[j];
  }
  if (s.mixed) {
    for (int64_t j = 0; j < ka; j++) s.rho_last[cl + j] = rho[j];
    // an FP32 iteration that did not halve the first column's residual: the
    // FP32 filter has reached its rounding floor there, and the columns after
    // it whose residuals are within an order of that one (or two orders of
    // the switch) are near the same floor, so they turn FP64 together (one
    // per iteration would cost an iteration each)
    if (s.prev_first32 && s.prev_first == cl && rho[0] > 0.5 * s.prev_first_rho) {
      const double floor_level = std::max(100.0 * s.mixed_switch * inf.h_H, 10.0 * rho[0]);
      int64_t j = cl + 1;
      while (j < s.k && s.rho_last[j] <= floor_level) j++;
      s.fp64_upto = std::max(s.fp64_upto, j);
    }
    s.prev_first = cl + nl;
    s.prev_first_rho = nl < ka ? rho[nl] : INFINITY;
    s.prev_first32 = nl < ka && nl >= s.split;  // that column's filter ran in FP32
  }
  s.cl += nl;
  s.a = mu[ka - 1];
  s.a0 = std::min(s.a0, mu[0]);
  inf.converged = (int32_t)s.cl;
  if (log_level() >= 2)
    std::fprintf(stderr,
                 "[chfsi] n=%lld it=%d locked=%lld/%lld active=%lld fp64_cols=%lld a=%.6g a0=%.6g b=%.6g "
                 "rho_first=%.3e (x h_H)\n",
                 (long long)n, s.it, (long long)s.cl, (long long)s.nev, (long long)ka, (long long)s.split, s.a, s.a0,
                 s.b, nl < ka ? rho[nl] / inf.h_H : 0.0);
  if (s.cl >= s.nev) {
    s.converged = true;
    s.done = true;
  } else if (s.it >= c->opts.max_iter) {
    s.done = true;
  }
}

void solve_finish(chfsi_ctx c, SolveState& s, chfsi_info* info) {
  const int64_t n = c->n;
  chfsi_info& inf = s.inf;
  inf.iterations = s.it;
  inf.a0 = s.a0;
  inf.a = s.a;
  const int64_t nout = s.converged ? s.nev : s.cl;
  double mx = 0.0;
  for (int64_t j = 0; j < s.nev; j++) {
    s.evals[j] = j < nout ? s.lam[j] : NAN;
    if (j < nout) mx = std::max(mx, s.rho_lock[j] / inf.h_H);
  }
  inf.max_rel_residual = mx;
  {
    Range r_back("chfsi.backtransform");
    if (s.X && s.nev > 0)
      c->gemm(OP_C, OP_N, n, s.nev, n, 1.0, c->Linv.z(), n, c->Y.z(), n, s.X, s.ldx, 0.0, nullptr, 0, 0.0, nullptr, 0,
              GEMM_TRI_A_UPPER);
    c->sync();
  }
  // warm state for the next problem of the sequence
  c->warm_valid = true;
  c->warm_k = s.k;
  c->warm_a0 = s.a0;
  c->warm_a = s.a;
  inf.filter_flops = c->filt_flops[0] + c->filt_flops[1];
  inf.filter_launches = c->filt_launches[0] + c->filt_launches[1];
  inf.filter_kernel_seconds = c->filt_kernel_s[0] + c->filt_kernel_s[1];
  inf.filter_flops_fp32 = c->filt_flops[1];
  inf.filter_launches_fp32 = c->filt_launches[1];
  inf.filter_kernel_seconds_fp32 = c->filt_kernel_s[1];
  inf.t_total = secs_since(s.t_start);
  if (log_level() >= 1)
    std::fprintf(stderr,
                 "[chfsi] solve n=%lld nev=%lld k=%lld precision=%d warm=%d iterations=%d (fp32 %d) locked=%d "
                 "t_total=%.4f s (reduce %.4f lanczos %.4f filter %.4f qr %.4f rr %.4f resid %.4f) "
                 "filter %.2f TFLOP max_rel_residual=%.3e\n",
                 (long long)n, (long long)s.nev, (long long)s.k, c->opts.precision, inf.warm_start, inf.iterations,
                 inf.iterations_fp32, inf.converged, inf.t_total, inf.t_reduce, inf.t_lanczos, inf.t_filter, inf.t_qr,
                 inf.t_rr, inf.t_resid, inf.filter_flops * 1e-12, inf.max_rel_residual);
  if (info) *info = inf;
  if (!s.converged)
    throw Error(ST_ENOCONV, "not converged after " + std::to_string(c->opts.max_iter) + " iterations (" +
                                std::to_string(s.cl) + " of " + std::to_string(s.nev) + " locked)");
}

// Run the whole of Algorithm 1.
void solve_impl(chfsi_ctx c, const zc* H, int64_t ldh, const zc* S, int64_t lds, int64_t nev, int64_t nex, const zc* Vw,
                int64_t ldv, int64_t kw, double tol, double* evals, zc* X, int64_t ldx, chfsi_info* info,
                const double* bounds_in = nullptr) {
  SolveState s;
  s.H = H; s.ldh = ldh; s.S = S; s.lds = lds; s.nev = nev; s.nex = nex; s.Vw = Vw; s.ldv = ldv; s.kw = kw;
  s.tol = tol; s.evals = evals; s.X = X; s.ldx = ldx; s.bounds_in = bounds_in;
  solve_begin(c, s);
  while (!s.done) {
    solve_filter(c, s);
    solve_post(c, s);
  }
  solve_finish(c, s, info);
}

}  // namespace

// ===========================================================================
// Serving: a request loop over many k-point sequences (Section 2: one
// sequence of correlated problems per k-point).  Worker threads each own a
// HIP stream and a solver context, so admitted solves overlap on the device;
// each sequence keeps its last block (generalized space) and filter bounds on
// the device to warm-start its next problem; requests are admitted while the
// device memory they need fits the budget.
// ===========================================================================
namespace {

struct SeqState {
  int64_t n = 0, k = 0;
  DBuf X;  // n x k block of the last solve, generalized space
  double a0 = 0, a = 0;
  bool valid = false, busy = false;
  // the overlap matrix of the sequence's last request that passed one (a
  // request without S reuses it: the factor of a worker that still holds
  // it, else a new factorization of this matrix)
  const zc* S = nullptr;
  int64_t lds = 0, S_n = 0;
};

struct Req {
  int64_t ticket = 0, seq = 0, n = 0, nev = 0, nex = 0;
  const zc* H = nullptr;
  int64_t ldh = 0;
  const zc* S = nullptr;
  int64_t lds = 0;
  double tol = 0;
  double* evals = nullptr;
  zc* X = nullptr;
  int64_t ldx = 0;
  std::chrono::steady_clock::time_point t_submit, t_end;
  int status = 0;
  bool done = false;
  chfsi_info info{};
  std::string err;
};

struct Worker {
  std::thread th;
  hipStream_t st = nullptr;
  chfsi_ctx ctx = nullptr;
  int64_t cap_n = 0, cap_k = 0;  // largest problem the context's buffers were grown for
  size_t bytes = 0;              // accounted footprint of ctx
  bool busy = false;
  bool recreate = false;  // next request: a fresh context of that request's size
  int64_t factor_seq = -1;  // sequence whose overlap factor the context holds
};

// Device bytes of a solver context for problems of size n with block k.
size_t ctx_footprint(int64_t n, int64_t k, int precision, int degree) {
  size_t z = sizeof(zc);
  size_t b = z * ((size_t)4 * n * n + (size_t)6 * n * k + (size_t)13 * k * k + (size_t)n * splitk_columns(k) +
                  (size_t)64 * n);
  if (precision >= 1) b += sizeof(cc) * ((size_t)n * n + (size_t)2 * n * k);
  if (precision >= 2) b += sizeof(cc) * (size_t)n * k + sizeof(double) * (size_t)(degree + 2) * k;
  if (precision == 3) b += (size_t)4 * n * f16_plane_ld(n) + (size_t)8 * k * f16_plane_ld(n);
  return b;
}

}  // namespace

struct chfsi_server_s {
  chfsi_server_config cfg{};
  int device = 0;
  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::unordered_map<int64_t, std::unique_ptr<Req>> reqs;
  std::unordered_map<int64_t, std::unique_ptr<SeqState>> seqs;
  std::vector<std::unique_ptr<Worker>> workers;
  size_t used = 0, peak = 0;
  bool stop = false;
  int64_t next_ticket = 1, submitted = 0, completed = 0, failed = 0, running = 0;
  std::vector<double> lat;
  bool have_first = false;
  std::chrono::steady_clock::time_point t_first, t_last;
  std::string err;

  size_t seq_need(const Req& r) const {
    auto it = seqs.find(r.seq);
    const int64_t k = r.nev + r.nex;
    const size_t want = (size_t)r.n * k * sizeof(zc);
    if (it == seqs.end()) return want;
    return it->second->X.bytes >= want ? 0 : want - it->second->X.bytes;
  }

  // Choose the next admissible request for worker w (lock held).  The
  // worker's context serves any problem its buffers were grown for; a larger
  // one grows it when the budget allows, else it is replaced by a context
  // of the request's size.  A request that reuses its sequence's overlap
  // factor goes to the idle worker holding that factor when there is one.
  Req* pick(Worker& w) {
    for (auto it = queue.begin(); it != queue.end(); ++it) {
      Req* r = *it;
      auto sq = seqs.find(r->seq);
      if (sq != seqs.end() && sq->second->busy) continue;  // one problem of a sequence at a time, in order
      const int64_t k = r->nev + r->nex;
      if (!r->S && w.factor_seq != r->seq) {
        bool holder_idle = false;
        for (auto& o : workers)
          if (o.get() != &w && !o->busy && o->factor_seq == r->seq && o->cap_n >= r->n && o->cap_k >= k)
            holder_idle = true;
        if (holder_idle) continue;
      }
      const size_t ctx_need = ctx_footprint(r->n, k, cfg.opts.precision, cfg.opts.degree);
      const size_t grown =
          ctx_footprint(std::max(w.cap_n, r->n), std::max(w.cap_k, k), cfg.opts.precision, cfg.opts.degree);
      size_t ctx_delta = w.ctx ? (grown > w.bytes ? grown - w.bytes : 0) : ctx_need;
      size_t ctx_freed = 0;
      bool recreate = false;
      size_t need = ctx_delta + seq_need(*r);
      if ((size_t)cfg.hbm_budget_bytes < ctx_need + (size_t)r->n * k * sizeof(zc)) {
        // can never fit
        r->status = CHFSI_ENOMEM;
        r->err = "request needs more device memory than the server budget";
        r->done = true;
        failed++;
        queue.erase(it);
        cv_done.notify_all();
        return pick(w);
      }
      if (used + need > (size_t)cfg.hbm_budget_bytes) {
        // release idle workers' contexts and retry
        for (auto& o : workers)
          if (o.get() != &w && !o->busy && o->ctx) {
            chfsi_release(o->ctx);
            o->ctx = nullptr;
            used -= o->bytes;
            o->bytes = 0;
            o->cap_n = o->cap_k = 0;
            o->factor_seq = -1;
          }
      }
      if (used + need > (size_t)cfg.hbm_budget_bytes && w.ctx && ctx_delta) {
        // this worker's own context replaced by one of the request's size
        recreate = true;
        ctx_freed = w.bytes;
        ctx_delta = ctx_need;
        need = ctx_delta + seq_need(*r);
      }
      if (used - ctx_freed + need > (size_t)cfg.hbm_budget_bytes) continue;
      queue.erase(it);
      used = used - ctx_freed + need;
      peak = std::max(peak, used);
      if (recreate) {
        w.recreate = true;
        w.bytes = ctx_need;
        w.cap_n = r->n;
        w.cap_k = k;
      } else if (ctx_delta || !w.ctx) {
        w.bytes = w.ctx ? grown : ctx_need;
        w.cap_n = std::max(w.cap_n, r->n);
        w.cap_k = std::max(w.cap_k, k);
      }
      auto& st = seqs[r->seq];
      if (!st) st.reset(new SeqState());
      st->busy = true;
      w.busy = true;
      running++;
      return r;
    }
    return nullptr;
  }

  void run(Worker& w, Req& r, SeqState& q) {
    const int64_t k = r.nev + r.nex;
    Range range("chfsi.server.request");
    try {
      if (w.recreate || !w.ctx) {
        if (w.ctx) chfsi_release(w.ctx);
        w.ctx = nullptr;
        w.recreate = false;
        w.factor_seq = -1;
        int st = chfsi_create(&w.ctx, r.n, &cfg.opts, w.st);
        if (st != CHFSI_OK) throw Error(st, "server: context creation failed");
      }
      chfsi_ctx c = w.ctx;
      c->resize(r.n);
      c->warm_valid = false;
      // the overlap matrix: the request's, else the factor this worker holds
      // for the sequence, else the sequence's remembered matrix
      const zc* S = r.S;
      int64_t lds = r.lds;
      if (S) {
        q.S = S;
        q.lds = lds;
        q.S_n = r.n;
      } else if (!(w.factor_seq == r.seq && c->have_factors)) {
        if (!q.S || q.S_n != r.n) throw Error(ST_EINVAL, "server: no overlap matrix for this sequence's request");
        S = q.S;
        lds = q.lds;
      }
      w.factor_seq = -1;  // until the reduction has run
      const bool warm = q.valid && q.n == r.n && q.k == k;
      const double bounds[2] = {q.a0, q.a};
      c->err.clear();
      solve_impl(c, r.H, r.ldh, S, lds, r.nev, r.nex, warm ? q.X.z() : nullptr, r.n, warm ? k : 0, r.tol, r.evals,
                 r.X, r.ldx, &r.info, warm ? bounds : nullptr);
      if (c->have_factors) w.factor_seq = r.seq;
      r.status = CHFSI_OK;
    } catch (const Error& e) {
      r.status = e.code;
      r.err = e.what();
      if (w.ctx && w.ctx->have_factors && e.code == ST_ENOCONV) w.factor_seq = r.seq;
    } catch (const std::exception& e) {
      r.status = CHFSI_EHIP;
      r.err = e.what();
    }
    // keep the block for the sequence's next problem (also after ENOCONV)
    if (r.status == CHFSI_OK || r.status == CHFSI_ENOCONV) {
      try {
        chfsi_ctx c = w.ctx;
        const int64_t n = r.n;
        q.X.ensure((size_t)n * k * sizeof(zc));
        c->gemm(OP_C, OP_N, n, k, n, 1.0, c->Linv.z(), n, c->Y.z(), n, q.X.z(), n, 0.0, nullptr, 0, 0.0, nullptr, 0,
                GEMM_TRI_A_UPPER);
        c->sync();
        q.n = n;
        q.k = k;
        q.a0 = c->warm_a0;
        q.a = c->warm_a;
        q.valid = true;
      } catch (const Error& e) {
        q.valid = false;
        if (r.status == CHFSI_OK) {
          r.status = e.code;
          r.err = e.what();
        }
      }
    } else {
      q.valid = false;
    }
  }
};

namespace {

void server_worker(chfsi_server s, Worker* w) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->m);
  while (true) {
    Req* r = nullptr;
    s->cv_work.wait(lk, [&] { return s->stop || (r = s->pick(*w)) != nullptr; });
    if (!r) break;  // stop requested and nothing admissible
    SeqState* q = s->seqs[r->seq].get();
    lk.unlock();
    s->run(*w, *r, *q);
    lk.lock();
    r->t_end = std::chrono::steady_clock::now();
    r->done = true;
    q->busy = false;
    w->busy = false;
    s->running--;
    if (r->status == CHFSI_OK) {
      s->completed++;
      s->lat.push_back(std::chrono::duration<double>(r->t_end - r->t_submit).count());
      s->t_last = r->t_end;
    } else {
      s->failed++;
      s->err = r->err;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
}

}  // namespace

// ===========================================================================
// Batching: Algorithm 1 for many independent problems in lockstep.  Each
// outer iteration runs the degree steps of every member's filter as grouped
// launches (one per step and precision), then each member's QR, Rayleigh-Ritz,
// residuals and locking on its own stream, issued from a few host threads.
// ===========================================================================
namespace {

// fn(i) for i in [0, count) on up to `threads` host threads, each with the
// device current; fn must not throw.
template <class F>
void for_members(int count, int threads, int device, F&& fn) {
  threads = std::max(1, std::min(threads, count));
  if (threads == 1) {
    for (int i = 0; i < count; i++) fn(i);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> th;
  th.reserve(threads);
  for (int t = 0; t < threads; t++)
    th.emplace_back([&] {
      (void)hipSetDevice(device);
      for (int i = next.fetch_add(1); i < count; i = next.fetch_add(1)) fn(i);
    });
  for (auto& x : th) x.join();
}

// Tile configurations the online choice tries, in order (11: the 64 x 64 x 16
// tile with eight waves, FP32 with four; 12: 64 x 80 x 16).
constexpr int BATCH_CANDIDATES[] = {3, 4, 5, 11, 7, 12};
constexpr int BATCH_NCAND = sizeof(BATCH_CANDIDATES) / sizeof(BATCH_CANDIDATES[0]);

}  // namespace

struct chfsi_batch_s {
  int count = 0;
  int device = 0;
  int threads = 8;
  bool use_graph = false;
  chfsi_opts opts{};
  std::vector<chfsi_ctx> mem;
  std::vector<hipStream_t> mst;
  std::vector<hipEvent_t> ready;
  hipStream_t gst = nullptr;  // the grouped launches
  hipEvent_t gdone = nullptr;
  hipEvent_t gt[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  // per precision: step parameters (degree x count, step-major) and tile
  // prefixes (degree x (count + 1)) on the device, with pinned staging
  DBuf gp[2], t0[2], ctr[2];  // ctr: 8 tile counters per degree step, zeroed before the steps
  DBuf e0[2];                 // per step, (count + 1) prefixes of the split members' elements
  ZGemmParams* hgp[2] = {nullptr, nullptr};
  int64_t* ht0[2] = {nullptr, nullptr};
  int64_t* he0[2] = {nullptr, nullptr};
  // online tile choice: chosen configuration (0 while trying), next trial,
  // measured rates
  int cfg[2] = {0, 0};
  int trial[2] = {0, 0};
  double rate[2][16] = {};
  int grid[2][16] = {};
  // captured degree steps per precision, for configuration gexec_cfg
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int gexec_cfg[2] = {0, 0};
  std::string err;

  void destroy() {
    for (int p = 0; p < 2; p++) {
      if (gexec[p]) (void)hipGraphExecDestroy(gexec[p]);
      gexec[p] = nullptr;
      if (hgp[p]) (void)hipHostFree(hgp[p]);
      if (ht0[p]) (void)hipHostFree(ht0[p]);
      if (he0[p]) (void)hipHostFree(he0[p]);
      he0[p] = nullptr;
      e0[p].release();
      hgp[p] = nullptr;
      ht0[p] = nullptr;
      gp[p].release();
      t0[p].release();
      ctr[p].release();
      for (int q = 0; q < 2; q++)
        if (gt[p][q]) (void)hipEventDestroy(gt[p][q]);
    }
    for (auto c : mem) chfsi_release(c);
    mem.clear();
    for (auto e : ready) (void)hipEventDestroy(e);
    ready.clear();
    for (auto x : mst) (void)hipStreamDestroy(x);
    mst.clear();
    if (gdone) (void)hipEventDestroy(gdone);
    if (gst) (void)hipStreamDestroy(gst);
    gdone = nullptr;
    gst = nullptr;
  }

  int grid_of(int prec, int c) {
    if (!grid[prec][c]) grid[prec][c] = zgemm_grouped_grid(prec, c);
    return grid[prec][c];
  }

  // Configuration for this iteration's steps in precision prec.
  int config_for(int prec) const { return cfg[prec] ? cfg[prec] : BATCH_CANDIDATES[trial[prec]]; }

  // The m grouped steps of precision prec on gst (parameters already on the device).
  void launch_steps(int prec, int c, int m) {
    const ZGemmParams* g = static_cast<const ZGemmParams*>(gp[prec].p);
    const int64_t* t = static_cast<const int64_t*>(t0[prec].p);
    int* cn = ctr[prec].i();
    fill_i32(cn, (int64_t)8 * m, 0, gst);  // a kernel, so it can sit in a captured graph
    const int64_t* el = static_cast<const int64_t*>(e0[prec].p);
    for (int i = 0; i < m; i++) {
      zgemm_grouped_filter_step(prec, c, g + (int64_t)i * count, t + (int64_t)i * (count + 1), count, cn + 8 * i,
                                grid_of(prec, c), gst);
      // split members' combination (no work when nothing was split)
      zgemm_grouped_reduce(prec, g + (int64_t)i * count, el + (int64_t)i * (count + 1), count, 1024, gst);
    }
  }

  void capture(int prec, int c, int m) {
    if (gexec[prec]) (void)hipGraphExecDestroy(gexec[prec]);
    gexec[prec] = nullptr;
    hipGraph_t graph = nullptr;
    (void)grid_of(prec, c);  // device queries stay outside the capture
    CHFSI_HIP(hipStreamBeginCapture(gst, hipStreamCaptureModeThreadLocal));
    try {
      launch_steps(prec, c, m);
    } catch (...) {
      (void)hipStreamEndCapture(gst, &graph);
      if (graph) (void)hipGraphDestroy(graph);
      throw;
    }
    CHFSI_HIP(hipStreamEndCapture(gst, &graph));
    hipError_t e = hipGraphInstantiate(&gexec[prec], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      gexec[prec] = nullptr;
      throw Error(ST_EHIP, std::string("graph instantiation failed: ") + hipGetErrorString(e));
    }
    gexec_cfg[prec] = c;
  }
};

namespace {

struct BatchMember {
  SolveState s;
  int status = CHFSI_OK;
  std::string err;
  bool active = false;     // taking part in the current iteration
  double iter_flops[2] = {0, 0};  // its filter flops per precision in the current iteration
  bool reuse = false;             // its FP64 first step came from W Z this iteration
  bool ritz = false;              // its FP32 range runs on the Ritz residual this iteration
};

void batch_solve_impl(chfsi_batch b, const void* const* H, const int64_t* ldh, const void* const* S,
                      const int64_t* lds, const int64_t* nev, const int64_t* nex, double tol, double* const* evals,
                      void* const* X, const int64_t* ldx, chfsi_info* infos, int32_t* statuses,
                      chfsi_batch_report* report) {
  const int G = b->count;
  check_ptr(H, "H");
  check_ptr(ldh, "ldh");
  check_ptr(nev, "nev");
  check_ptr(nex, "nex");
  check_ptr(evals, "evals");
  check_ptr(infos, "infos");
  check_ptr(statuses, "statuses");
  if (S) check_ptr(lds, "lds");
  if (X) check_ptr(ldx, "ldx");
  if (!(tol > 0.0)) throw Error(ST_EINVAL, "tol must be positive");
  for (int j = 0; j < G; j++) {
    const int64_t n = b->mem[j]->n;
    const std::string w = " (member " + std::to_string(j) + ")";
    if (!H[j]) throw Error(ST_EINVAL, "null H" + w);
    if (!evals[j]) throw Error(ST_EINVAL, "null evals" + w);
    if (!block_sizes_ok(n, nev[j], nex[j])) throw Error(ST_EINVAL, BLOCK_SIZES_RULE + w);
    if (ldh[j] < n) throw Error(ST_EINVAL, "ldh smaller than n" + w);
    if (S && S[j] && lds[j] < n) throw Error(ST_EINVAL, "lds smaller than n" + w);
    if (X && X[j] && ldx[j] < n) throw Error(ST_EINVAL, "ldx smaller than n" + w);
  }
  const auto t_start = std::chrono::steady_clock::now();
  CHFSI_HIP(hipDeviceSynchronize());  // callers' inputs are complete

  chfsi_batch_report rep{};
  const int m = b->opts.degree;
  std::vector<std::unique_ptr<BatchMember>> mb(G);
  for (int j = 0; j < G; j++) {
    mb[j].reset(new BatchMember());
    SolveState& s = mb[j]->s;
    s.H = static_cast<const zc*>(H[j]);
    s.ldh = ldh[j];
    s.S = S ? static_cast<const zc*>(S[j]) : nullptr;
    s.lds = S ? lds[j] : 0;
    s.nev = nev[j];
    s.nex = nex[j];
    s.tol = tol;
    s.evals = evals[j];
    s.X = X ? static_cast<zc*>(X[j]) : nullptr;
    s.ldx = X ? ldx[j] : 0;
  }
  auto fail = [&](int j, const Error& e) {
    mb[j]->status = e.code;
    mb[j]->err = e.what();
    mb[j]->s.done = true;
    (void)hipGetLastError();
  };
  auto member_guard = [&](int j, auto&& f) {
    try {
      f();
    } catch (const Error& e) {
      fail(j, e);
    } catch (const std::exception& e) {
      fail(j, Error(ST_EHIP, e.what()));
    }
  };

  // reduction, bounds and start blocks
  for_members(G, b->threads, b->device, [&](int j) {
    member_guard(j, [&] {
      b->mem[j]->err.clear();
      solve_begin(b->mem[j], mb[j]->s);
    });
  });

  for (int it = 0;; it++) {
    // active members; act[p]: those with columns filtered in precision p
    // (FP64: the leading `split` active columns, FP32: the rest)
    std::vector<int> all, act[2];
    for (int j = 0; j < G; j++) {
      mb[j]->active = !mb[j]->s.done;
      if (!mb[j]->active) continue;
      SolveState& s = mb[j]->s;
      solve_filter_begin(s);
      all.push_back(j);
      if (s.split > 0) act[0].push_back(j);
      if (s.split < s.k - s.cl) act[1].push_back(j);
    }
    if (all.empty()) break;
    rep.outer_iterations++;
    // first column and width of member j's range in precision p
    auto range = [&](int j, int p, int64_t& c0, int64_t& w) {
      const SolveState& s = mb[j]->s;
      c0 = p ? s.cl + s.split : s.cl;
      w = p ? s.k - s.cl - s.split : s.split;
    };

    // members' blocks ready for the grouped steps
    for (int j : all) {
      chfsi_ctx c = b->mem[j];
      SolveState& s = mb[j]->s;
      const int64_t n = c->n;
      int64_t c32, w32;
      range(j, 1, c32, w32);
      CHFSI_HIP(hipEventRecord(s.ev[0], c->st));
      // precision 2 with Ritz vectors at hand: the Ritz-residual form (its
      // first step needs no product), else the block rounded to FP32
      mb[j]->ritz = s.ritz && w32 > 0 && s.wz_first >= 0 && s.cl >= s.wz_first;
      if (mb[j]->ritz)
        c->ritz_prepare(c->Y.z() + c32 * n, n, c->Wz.z() + (c32 - s.wz_first) * n, n,
                        c->mu.d() + (c32 - s.wz_first), s.lam.data() + c32, w32, cheb_schedule(m, s.a, s.b, s.a0),
                        (cc*)c->Y32b.p);
      else if (w32 > 0)
        to_f32(c->Y.z() + c32 * n, n, (cc*)c->Y32.p, n, n, w32, c->st);
      // the FP64 range's first step from the last Rayleigh-Ritz product W Z = A Y
      mb[j]->reuse = s.split > 0 && s.wz_first >= 0 && s.cl >= s.wz_first;
      if (mb[j]->reuse) {
        const ChebStep c0 = cheb_schedule(1, s.a, s.b, s.a0)[0];
        lincomb2d(c0.alpha, c->Wz.z() + (s.cl - s.wz_first) * n, n, c0.beta, c->Y.z() + s.cl * n, n,
                  c->Yb.z() + s.cl * n, n, n, s.split, c->st);
      }
      CHFSI_HIP(hipEventRecord(b->ready[j], c->st));
      CHFSI_HIP(hipStreamWaitEvent(b->gst, b->ready[j], 0));
      mb[j]->iter_flops[0] = mb[j]->iter_flops[1] = 0.0;
    }

    double flops[2] = {0, 0};
    int used_cfg[2] = {0, 0};
    for (int p = 0; p < 2; p++) {
      if (act[p].empty()) continue;
      const int cf = b->config_for(p);
      used_cfg[p] = cf;
      int bm = 0, bn = 0;
      zgemm_tile_shape(cf, &bm, &bn);
      ZGemmParams* hp = b->hgp[p];
      int64_t* ht = b->ht0[p];
      std::vector<char> on(G, 0);
      for (int j : act[p]) on[j] = 1;
      int64_t* he = b->he0[p];
      for (int i = 0; i < m; i++) ht[(int64_t)i * (G + 1)] = he[(int64_t)i * (G + 1)] = 0;
      const int bk = zgemm_config_bk(cf);
      for (int j = 0; j < G; j++) {
        int64_t tiles = 0, elems = 0;
        bool skip0 = false;  // step 0 done without a product (reuse of W Z)
        if (on[j]) {
          chfsi_ctx c = b->mem[j];
          const SolveState& s = mb[j]->s;
          const int64_t n = c->n;
          int64_t c0, w;
          range(j, p, c0, w);
          const int64_t tm = cdiv(n, (int64_t)bm), tn = cdiv(w, (int64_t)bn);
          // K split as in single solves (chunks near 1000 deep), within the
          // member's partial-tile buffer
          int sk = (int)std::min<int64_t>(4, std::max<int64_t>(1, (n + 500) / 1000));
          const size_t cap = c->P_elems * (p ? 2 : 1);
          while (sk > 1 && ((size_t)sk * n * w > cap || n < (int64_t)sk * 4 * bk)) sk--;
          const int64_t kchunk = cdiv(cdiv(n, (int64_t)sk), (int64_t)bk) * bk;
          sk = (int)cdiv(n, kchunk);
          tiles = tm * tn * sk;
          elems = sk > 1 ? n * w : 0;
          char* y0 = p ? (char*)c->Y32.p : (char*)(c->Y.z() + c0 * n);
          char* y1 = p ? (char*)c->Y32b.p : (char*)(c->Yb.z() + c0 * n);
          const std::vector<ChebStep> cs = cheb_schedule(m, s.a, s.b, s.a0);
          const bool ritz = p == 1 && mb[j]->ritz;  // D_1 already in y1, D_0 = 0
          void *cur = y0, *out = y1;
          for (int i = 0; i < m; i++) {
            ZGemmParams q{};
            q.M = n; q.N = w; q.K = n;
            q.A = p ? c->A32.p : (const void*)c->A.z(); q.lda = n;
            q.B = cur; q.ldb = n;
            q.C = out; q.ldc = n;
            q.X = cur; q.ldx = n;
            q.Z = i && !(ritz && i == 1) ? out : nullptr; q.ldz = n;
            if (ritz && i > 0) {
              q.R = c->R32.p; q.ldr = n;
              q.rs = c->ctab.d() + (size_t)i * w;
            }
            q.alpha = cs[i].alpha; q.beta = cs[i].beta; q.gamma = cs[i].gamma;
            q.flags = 0; q.splitk = sk; q.kchunk = sk > 1 ? kchunk : n; q.P = sk > 1 ? c->P.p : nullptr;
            q.tiles_m = (int)tm; q.tiles_n = (int)tn;
            hp[(int64_t)i * G + j] = q;
            std::swap(cur, out);
          }
          skip0 = (p == 0 && mb[j]->reuse) || ritz;
          const int products = skip0 ? m - 1 : m;
          const double f = 8.0 * (double)n * (double)n * (double)w * (double)products;
          mb[j]->iter_flops[p] = f;
          flops[p] += f;
          c->filt_launches[p] += products;
          c->filt_flops[p] += f;
        } else {
          for (int i = 0; i < m; i++) hp[(int64_t)i * G + j] = ZGemmParams{};
        }
        for (int i = 0; i < m; i++) {
          int64_t* hi = ht + (int64_t)i * (G + 1);
          int64_t* hq = he + (int64_t)i * (G + 1);
          const bool none = i == 0 && skip0;
          hi[j + 1] = hi[j] + (none ? 0 : tiles);
          hq[j + 1] = hq[j] + (none ? 0 : elems);
        }
      }
      CHFSI_HIP(hipMemcpyAsync(b->gp[p].p, hp, (size_t)m * G * sizeof(ZGemmParams), hipMemcpyHostToDevice, b->gst));
      CHFSI_HIP(hipMemcpyAsync(b->t0[p].p, ht, (size_t)m * (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice, b->gst));
      CHFSI_HIP(hipMemcpyAsync(b->e0[p].p, he, (size_t)m * (G + 1) * sizeof(int64_t), hipMemcpyHostToDevice, b->gst));
      CHFSI_HIP(hipEventRecord(b->gt[p][0], b->gst));
      const bool graph = b->use_graph && b->cfg[p] != 0;
      if (graph) {
        if (!b->gexec[p] || b->gexec_cfg[p] != cf) b->capture(p, cf, m);
        CHFSI_HIP(hipGraphLaunch(b->gexec[p], b->gst));
        rep.graph = 1;
      } else {
        b->launch_steps(p, cf, m);
      }
      CHFSI_HIP(hipEventRecord(b->gt[p][1], b->gst));
      rep.grouped_launches += m;
    }
    CHFSI_HIP(hipEventRecord(b->gdone, b->gst));

    // results into F(:, cl:k), then each member's QR / Rayleigh-Ritz / locking
    for (int j : all) {
      chfsi_ctx c = b->mem[j];
      SolveState& s = mb[j]->s;
      const int64_t n = c->n;
      CHFSI_HIP(hipStreamWaitEvent(c->st, b->gdone, 0));
      int64_t c0, w;
      range(j, 0, c0, w);
      if (w > 0) {
        const zc* r = (m & 1) ? c->Yb.z() + c0 * n : c->Y.z() + c0 * n;
        copy2d(r, n, c->F.z() + c0 * n, n, n, w, c->st);
      }
      range(j, 1, c0, w);
      if (w > 0) {
        const cc* r = (const cc*)((m & 1) ? c->Y32b.p : c->Y32.p);
        if (mb[j]->ritz) c->ritz_finish(c->Y.z() + c0 * n, n, r, m, w, c->F.z() + c0 * n, n);
        else to_f64(r, n, c->F.z() + c0 * n, n, n, w, c->st);
        s.inf.iterations_fp32++;
      }
      CHFSI_HIP(hipEventRecord(s.ev[1], c->st));
    }
    for_members((int)all.size(), b->threads, b->device, [&](int q) {
      const int j = all[q];
      member_guard(j, [&] { solve_post(b->mem[j], mb[j]->s); });
    });

    // grouped step times (every member stream has passed gdone)
    CHFSI_HIP(hipEventSynchronize(b->gdone));
    for (int p = 0; p < 2; p++) {
      if (act[p].empty()) continue;
      float ms = 0.f;
      CHFSI_HIP(hipEventElapsedTime(&ms, b->gt[p][0], b->gt[p][1]));
      const double sec = ms * 1e-3;
      rep.filter_seconds += sec;
      rep.filter_flops += flops[p];
      // members' share of the launch time, in proportion to their flops
      for (int j : act[p])
        if (flops[p] > 0) b->mem[j]->filt_kernel_s[p] += sec * mb[j]->iter_flops[p] / flops[p];
      if (!b->cfg[p]) {
        const int cf = used_cfg[p];
        if (sec > 0) b->rate[p][cf] = flops[p] / sec * 1e-12;
        b->trial[p]++;
        if (b->trial[p] >= BATCH_NCAND) {
          int best = BATCH_CANDIDATES[0];
          for (int q = 0; q < BATCH_NCAND; q++)
            if (b->rate[p][BATCH_CANDIDATES[q]] > b->rate[p][best]) best = BATCH_CANDIDATES[q];
          // near ties (within 2 % of the best rate): the narrower tile, which
          // pads less as the active widths shrink in later iterations (the
          // trials run on the first iterations of a cold start)
          const double top = b->rate[p][best];
          int bm = 0, bn_best = 0;
          zgemm_tile_shape(best, &bm, &bn_best);
          for (int q = 0; q < BATCH_NCAND; q++) {
            const int cq = BATCH_CANDIDATES[q];
            int bn = 0;
            zgemm_tile_shape(cq, &bm, &bn);
            if (bn < bn_best && b->rate[p][cq] >= 0.98 * top) {
              best = cq;
              bn_best = bn;
            }
          }
          b->cfg[p] = best;
        }
      }
    }
  }

  for_members(G, b->threads, b->device, [&](int j) {
    if (mb[j]->status != CHFSI_OK) return;
    member_guard(j, [&] { solve_finish(b->mem[j], mb[j]->s, &infos[j]); });
  });
  int first_bad = -1;
  for (int j = 0; j < G; j++) {
    statuses[j] = mb[j]->status;
    if (mb[j]->status == CHFSI_OK) rep.converged_members++;
    else if (first_bad < 0) first_bad = j;
    if (mb[j]->status != CHFSI_OK && mb[j]->status != CHFSI_ENOCONV) {
      infos[j] = mb[j]->s.inf;
      b->mem[j]->warm_valid = false;
    }
  }
  for (auto x : b->mst) CHFSI_HIP(hipStreamSynchronize(x));
  CHFSI_HIP(hipStreamSynchronize(b->gst));
  rep.tile_config = b->cfg[0] ? b->cfg[0] : 0;
  rep.tile_config_fp32 = b->cfg[1] ? b->cfg[1] : 0;
  for (int q = 0; q < 16; q++) rep.tile_rate[q] = b->rate[0][q];
  rep.seconds = secs_since(t_start);
  if (report) *report = rep;
  if (first_bad >= 0)
    throw Error(mb[first_bad]->status, "member " + std::to_string(first_bad) + ": " + mb[first_bad]->err);
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free GEMM (chfsi_zgemm_static): its split-K partial tiles live
// in this fixed array, one copy per GPU, held until the process ends.  Host
// code never passes the array's name to a kernel or a copy (on the host it is
// only a stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
// ---------------------------------------------------------------------------
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)64 << 20;  // CHFSI_STATIC_SCRATCH_BYTES in chfsi.h
static __device__ __align__(256) double scratch[STATIC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_static_mu;
void* g_static_ptr[STATIC_MAX_DEVICES] = {};
thread_local std::string g_static_err;

// Argument checks shared by chfsi_zgemm and chfsi_zgemm_static (throws
// CHFSI_EINVAL); false when the product is empty (nothing to launch).
bool zgemm_args_ok(int32_t opA, int32_t opB, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B,
                   int64_t ldb, const void* X, int64_t ldx, const void* Z, int64_t ldz, const void* C, int64_t ldc,
                   int32_t flags) {
  const int cfg = (flags >> 8) & 0xff;
  if (M < 0 || N < 0 || K < 0 || (opA != 0 && opA != 1) || (opB != 0 && opB != 1) || (flags & 0xff0000e0) ||
      cfg >= zgemm_num_configs())
    throw Error(ST_EINVAL, "zgemm: bad sizes, ops or flags");
  if (M == 0 || N == 0) return false;
  check_ptr(C, "C");
  check_ld(ldc, M, "ldc");
  if (K > 0) {
    check_ptr(A, "A");
    check_ptr(B, "B");
    check_ld(lda, opA == 0 ? M : K, "lda");
    check_ld(ldb, opB == 0 ? K : N, "ldb");
  }
  if (X) check_ld(ldx, M, "ldx");
  if (Z) check_ld(ldz, M, "ldz");
  return true;
}

// Device address of `scratch` on the current device (looked up on the first
// call per device).
void* static_scratch_ptr() {
  int dev = -1;
  CHFSI_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= STATIC_MAX_DEVICES) throw Error(ST_EHIP, "static scratch: device index out of range");
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      throw Error(ST_EHIP, std::string("static scratch: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
    }
    g_static_ptr[dev] = p;
  }
  return g_static_ptr[dev];
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void chfsi_default_opts(chfsi_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->degree = 20;
  o->max_iter = 1000;
  o->lanczos_steps = 10;
  o->precision = 0;
  o->seed = 0;
  o->profile = 0;
  o->qr_mode = 0;
}

const char* chfsi_status_string(chfsi_status s) {
  switch (s) {
    case CHFSI_OK: return "CHFSI_OK";
    case CHFSI_EINVAL: return "CHFSI_EINVAL";
    case CHFSI_ENOTPD: return "CHFSI_ENOTPD";
    case CHFSI_ENOCONV: return "CHFSI_ENOCONV";
    case CHFSI_ENAN: return "CHFSI_ENAN";
    case CHFSI_ENOMEM: return "CHFSI_ENOMEM";
    case CHFSI_EHIP: return "CHFSI_EHIP";
  }
  return "unknown";
}

chfsi_status chfsi_create(chfsi_ctx* out, int64_t n, const chfsi_opts* opts, void* stream) {
  if (!out) return CHFSI_EINVAL;
  *out = nullptr;
  if (n < 1) return CHFSI_EINVAL;
  chfsi_opts o;
  chfsi_default_opts(&o);
  if (opts) o = *opts;
  if (o.degree < 1 || o.max_iter < 1 || o.lanczos_steps < 1 || o.lanczos_steps > JACOBI_LDS_MAX || o.precision < 0 || o.precision > 3 ||
      (o.qr_mode != 0 && o.qr_mode != 1) || o.filter_tile < 0 || o.filter_tile >= zgemm_num_configs() ||
      o.filter_splitk < 0 || o.filter_splitk > 16 || o.mixed_switch_digits < 0 || o.mixed_switch_digits > 12)
    return CHFSI_EINVAL;
  chfsi_ctx c = new (std::nothrow) chfsi_ctx_s();
  if (!c) return CHFSI_ENOMEM;
  c->n = n;
  c->opts = o;
  c->st = (hipStream_t)stream;
  *out = c;
  return CHFSI_OK;
}

void chfsi_release(chfsi_ctx c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->st);
  c->free_all();
  delete c;
}

const char* chfsi_last_error(chfsi_ctx c) {
  if (c) return c->err.c_str();
  return g_static_err.empty() ? "null context" : g_static_err.c_str();
}

chfsi_status chfsi_reset(chfsi_ctx c) {
  return guarded(c, [&] { c->warm_valid = false; });
}

chfsi_status chfsi_reduce(chfsi_ctx c, const void* H, int64_t ldh, const void* S, int64_t lds) {
  return guarded(c, [&] {
    check_ptr(H, "H");
    check_ld(ldh, c->n, "ldh");
    if (S) check_ld(lds, c->n, "lds");
    c->reduce((const zc*)H, ldh, (const zc*)S, lds);
    c->sync();
  });
}

chfsi_status chfsi_solve(chfsi_ctx c, const void* H, int64_t ldh, const void* S, int64_t lds, int64_t nev, int64_t nex,
                         const void* V_warm, int64_t ldv, int64_t kw, double tol, double* evals, void* X, int64_t ldx,
                         chfsi_info* info) {
  return guarded(c, [&] {
    solve_impl(c, (const zc*)H, ldh, (const zc*)S, lds, nev, nex, (const zc*)V_warm, ldv, kw, tol, evals, (zc*)X, ldx,
               info);
  });
}

chfsi_status chfsi_copy_factors(chfsi_ctx c, void* A, int64_t lda, void* L, int64_t ldl, void* Linv, int64_t ldi) {
  return guarded(c, [&] {
    if (!c->have_factors) throw Error(ST_EINVAL, "no factors: call chfsi_reduce first");
    const int64_t n = c->n;
    if (A) { check_ld(lda, n, "lda"); copy2d(c->A.z(), n, (zc*)A, lda, n, n, c->st); }
    if (L) { check_ld(ldl, n, "ldl"); copy2d(c->L.z(), n, (zc*)L, ldl, n, n, c->st); }
    if (Linv) { check_ld(ldi, n, "ldi"); copy2d(c->Linv.z(), n, (zc*)Linv, ldi, n, n, c->st); }
    c->sync();
  });
}

chfsi_status chfsi_filter(chfsi_ctx c, const void* A, int64_t lda, void* Y, int64_t ldy, int64_t k, int32_t m, double a,
                          double b, double a0) {
  return guarded(c, [&] {
    check_ptr(A, "A");
    check_ptr(Y, "Y");
    check_ld(lda, c->n, "lda");
    check_ld(ldy, c->n, "ldy");
    if (k < 1 || k > c->n || m < 1 || !(b > a)) throw Error(ST_EINVAL, "filter: need 1 <= k <= n, m >= 1, b > a");
    c->ensure_small();
    c->ensure_k(k);
    c->reset_filter_stats();
    if (c->opts.filter_splitk > 1 && c->P_elems < (size_t)c->opts.filter_splitk * c->n * k) {
      c->P_elems = (size_t)c->opts.filter_splitk * c->n * k;
      c->P.release();
      c->P.ensure(c->P_elems * sizeof(zc));
    }
    c->P_cap = std::max(c->P_cap, std::min(c->P_elems, (size_t)c->opts.filter_splitk * c->n * k));
    const int64_t n = c->n;
    if (c->opts.precision >= 1) {
      // mixed precision: the filter itself in complex FP32 (no Ritz values
      // here: the plain recurrence)
      c->A32.ensure((size_t)n * n * sizeof(cc));
      c->Y32.ensure((size_t)n * k * sizeof(cc));
      c->Y32b.ensure((size_t)n * k * sizeof(cc));
      to_f32((const zc*)A, lda, (cc*)c->A32.p, n, n, n, c->st);
      to_f32((const zc*)Y, ldy, (cc*)c->Y32.p, n, n, k, c->st);
      void* r = c->filter_any(PREC_F32, c->A32.p, n, c->Y32.p, n, c->Y32b.p, n, k, m, a, b, a0);
      to_f64((const cc*)r, n, (zc*)Y, ldy, n, k, c->st);
    } else {
      zc* res = c->filter((const zc*)A, lda, (zc*)Y, ldy, c->Yb.z(), n, k, m, a, b, a0);
      if (res != (zc*)Y) copy2d(res, n, (zc*)Y, ldy, n, k, c->st);
    }
    c->sync();
    c->collect_filter_events();
  });
}

chfsi_status chfsi_filter_ritz(chfsi_ctx c, const void* A, int64_t lda, void* Y, int64_t ldy, const void* AY,
                               int64_t lday, const double* mu, int64_t k, int32_t m, double a, double b, double a0) {
  return guarded(c, [&] {
    check_ptr(A, "A");
    check_ptr(Y, "Y");
    check_ptr(AY, "AY");
    check_ptr(mu, "mu");
    check_ld(lda, c->n, "lda");
    check_ld(ldy, c->n, "ldy");
    check_ld(lday, c->n, "lday");
    if (k < 1 || k > c->n || m < 1 || !(b > a)) throw Error(ST_EINVAL, "filter: need 1 <= k <= n, m >= 1, b > a");
    c->ensure_small();
    c->ensure_k(k);
    c->reset_filter_stats();
    if (c->opts.filter_splitk > 1 && c->P_elems < (size_t)c->opts.filter_splitk * c->n * k) {
      c->P_elems = (size_t)c->opts.filter_splitk * c->n * k;
      c->P.release();
      c->P.ensure(c->P_elems * sizeof(zc));
    }
    c->P_cap = std::max(c->P_cap, std::min(c->P_elems, (size_t)c->opts.filter_splitk * c->n * k));
    const int64_t n = c->n;
    c->Y32.ensure((size_t)n * k * sizeof(cc));
    c->Y32b.ensure((size_t)n * k * sizeof(cc));
    c->R32.ensure((size_t)n * k * sizeof(cc));
    const bool half = c->opts.precision == 3;
    if (half) {
      c->A16.ensure((size_t)2 * n * f16_plane_ld(n) * sizeof(_Float16));
      to_f16_planes((const zc*)A, lda, n, c->A16.p, c->st);
    } else {
      c->A32.ensure((size_t)n * n * sizeof(cc));
      to_f32((const zc*)A, lda, (cc*)c->A32.p, n, n, n, c->st);
    }
    std::vector<double> mu_h(mu, mu + k);
    CHFSI_HIP(hipMemcpyAsync(c->mu.p, mu_h.data(), k * sizeof(double), hipMemcpyHostToDevice, c->st));
    c->filter_ritz((const zc*)Y, ldy, (const zc*)AY, lday, c->mu.d(), mu_h.data(), k, m, a, b, a0, c->F.z(), n, half);
    copy2d(c->F.z(), n, (zc*)Y, ldy, n, k, c->st);
    c->sync();
    c->collect_filter_events();
  });
}

chfsi_status chfsi_qr(chfsi_ctx c, void* Y, int64_t ldy, int64_t k) {
  return guarded(c, [&] {
    check_ptr(Y, "Y");
    check_ld(ldy, c->n, "ldy");
    if (k < 1 || k > c->n) throw Error(ST_EINVAL, "qr: need 1 <= k <= n");
    c->ensure_small();
    c->ensure_k(k);
    copy2d((zc*)Y, ldy, c->F.z(), c->n, c->n, k, c->st);
    c->qr(c->F.z(), c->n, k, (zc*)Y, ldy);
    c->sync();
  });
}

chfsi_status chfsi_orthonormalize(chfsi_ctx c, void* Y, int64_t ldy, int64_t k, int32_t* used_householder) {
  return guarded(c, [&] {
    check_ptr(Y, "Y");
    check_ld(ldy, c->n, "ldy");
    if (k < 1 || k > c->n) throw Error(ST_EINVAL, "orthonormalize: need 1 <= k <= n");
    c->ensure_small();
    c->ensure_k(k);
    copy2d((zc*)Y, ldy, c->F.z(), c->n, c->n, k, c->st);
    const bool hh = c->orthonormalize(c->F.z(), k, (zc*)Y, ldy);
    c->sync();
    if (used_householder) *used_householder = hh ? 1 : 0;
  });
}

chfsi_status chfsi_eigh(chfsi_ctx c, const void* G, int64_t ldg, int64_t k, double* w, void* Z, int64_t ldz) {
  return guarded(c, [&] {
    check_ptr(G, "G");
    check_ptr(w, "w");
    check_ptr(Z, "Z");
    if (k < 1) throw Error(ST_EINVAL, "eigh: k < 1");
    check_ld(ldg, k, "ldg");
    check_ld(ldz, k, "ldz");
    // the eigensolver's k x k scratch lives in the n x k block buffers
    if (k > c->n) throw Error(ST_EINVAL, "eigh: k > n of the context");
    c->ensure_small();
    c->ensure_k(k);
    c->refine_ok_last = false;  // no speculation across separate calls
    c->eigh((const zc*)G, ldg, k, c->mu.d(), (zc*)Z, ldz);
    c->ensure_host((size_t)k + 16);
    CHFSI_HIP(hipMemcpyAsync(c->hbuf, c->mu.p, k * sizeof(double), hipMemcpyDeviceToHost, c->st));
    c->sync();
    std::memcpy(w, c->hbuf, k * sizeof(double));
  });
}

chfsi_status chfsi_rayleigh_ritz(chfsi_ctx c, const void* A, int64_t lda, void* Y, int64_t ldy, int64_t k, double* mu) {
  return guarded(c, [&] {
    check_ptr(A, "A");
    check_ptr(Y, "Y");
    check_ptr(mu, "mu");
    check_ld(lda, c->n, "lda");
    check_ld(ldy, c->n, "ldy");
    if (k < 1 || k > c->n) throw Error(ST_EINVAL, "rayleigh_ritz: need 1 <= k <= n");
    c->ensure_small();
    c->ensure_k(k);
    copy2d((zc*)Y, ldy, c->Qb.z(), c->n, c->n, k, c->st);
    c->refine_ok_last = false;  // no speculation across separate calls
    c->rayleigh_ritz((const zc*)A, lda, c->Qb.z(), c->n, k, (zc*)Y, ldy, c->mu.d(), c->Wk.z(), nullptr);
    CHFSI_HIP(hipMemcpyAsync(c->hbuf, c->mu.p, k * sizeof(double), hipMemcpyDeviceToHost, c->st));
    c->sync();
    std::memcpy(mu, c->hbuf, k * sizeof(double));
  });
}

chfsi_status chfsi_residuals(chfsi_ctx c, const void* A, int64_t lda, const void* L, int64_t ldl, const void* Y,
                             int64_t ldy, int64_t k, const double* mu, double* rho) {
  return guarded(c, [&] {
    check_ptr(A, "A");
    check_ptr(L, "L");
    check_ptr(Y, "Y");
    check_ptr(mu, "mu");
    check_ptr(rho, "rho");
    check_ld(lda, c->n, "lda");
    check_ld(ldl, c->n, "ldl");
    check_ld(ldy, c->n, "ldy");
    if (k < 1 || k > c->n) throw Error(ST_EINVAL, "residuals: need 1 <= k <= n");
    c->ensure_small();
    c->ensure_k(k);
    const int64_t n = c->n;
    std::memcpy(c->hbuf, mu, k * sizeof(double));
    CHFSI_HIP(hipMemcpyAsync(c->mu.p, c->hbuf, k * sizeof(double), hipMemcpyHostToDevice, c->st));
    c->gemm(OP_N, OP_N, n, k, n, 1.0, (const zc*)A, lda, (const zc*)Y, ldy, c->Wz.z(), n);
    c->residual_norms((const zc*)L, ldl, c->Wz.z(), (const zc*)Y, ldy, k, c->mu.d(), c->Wk.z(), c->F.z(), c->rho.d());
    CHFSI_HIP(hipMemcpyAsync(c->hbuf + k, c->rho.p, k * sizeof(double), hipMemcpyDeviceToHost, c->st));
    c->sync();
    std::memcpy(rho, c->hbuf + k, k * sizeof(double));
  });
}

chfsi_status chfsi_lanczos(chfsi_ctx c, const void* A, int64_t lda, int32_t steps, uint64_t seed, uint32_t stream_id,
                           double* out) {
  return guarded(c, [&] {
    check_ptr(A, "A");
    check_ptr(out, "out");
    check_ld(lda, c->n, "lda");
    if (steps < 1 || steps > JACOBI_LDS_MAX) throw Error(ST_EINVAL, "lanczos: steps out of range");
    c->ensure_small();
      chfsi_opts keep = c->opts;
    c->opts.lanczos_steps = std::max(c->opts.lanczos_steps, steps);
    c->ensure_small();
    c->opts = keep;
    c->lanczos((const zc*)A, lda, steps, seed, stream_id, out);
  });
}

chfsi_status chfsi_random_block(chfsi_ctx c, uint64_t seed, uint32_t stream_id, int64_t col0, void* Y, int64_t ldy,
                                int64_t k) {
  return guarded(c, [&] {
    check_ptr(Y, "Y");
    check_ld(ldy, c->n, "ldy");
    if (k < 0 || col0 < 0) throw Error(ST_EINVAL, "random_block: negative size");
    random_block(seed, stream_id, c->n, k, col0, (zc*)Y, ldy, c->st);
    c->sync();
  });
}

chfsi_status chfsi_philox(chfsi_ctx c, const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count) {
  return guarded(c, [&] {
    if (count < 0) throw Error(ST_EINVAL, "philox: count < 0");
    if (count > 0) {
      check_ptr(ctr, "ctr");
      check_ptr(key, "key");
      check_ptr(out, "out");
    }
    philox_raw(ctr, key, out, count, c->st);
    c->sync();
  });
}

chfsi_status chfsi_zgemm(chfsi_ctx c, int32_t opA, int32_t opB, int64_t M, int64_t N, int64_t K, double alpha,
                         const void* A, int64_t lda, const void* B, int64_t ldb, double beta, const void* X, int64_t ldx,
                         double gamma, const void* Z, int64_t ldz, void* C, int64_t ldc, int32_t flags) {
  return guarded(c, [&] {
    const int structure = flags & 31, cfg = (flags >> 8) & 0xff, nsplit = (flags >> 16) & 0xff;
    if (!zgemm_args_ok(opA, opB, M, N, K, A, lda, B, ldb, X, ldx, Z, ldz, C, ldc, flags)) return;
    c->ensure_small();
    // split-K scratch: the requested split, or 16-way for small outputs
    size_t need = (cdiv(M, 32) * cdiv(N, 32) < 256) ? (size_t)M * N * 16 : 0;
    if (nsplit > 1) need = std::max(need, (size_t)M * N * nsplit);
    if (need && c->P_elems < need) {
      c->P.release();
      c->P.ensure(need * sizeof(zc));
      c->P_elems = need;
    }
    c->P_cap = c->P_elems;  // this product may use the whole scratch
    c->gemm(opA, opB, M, N, K, alpha, (const zc*)A, lda, (const zc*)B, ldb, (zc*)C, ldc, beta, (const zc*)X, ldx, gamma,
            (const zc*)Z, ldz, structure, true, false, cfg, nsplit);
    c->sync();
  });
}

chfsi_status chfsi_zgemm_static(void* stream, int32_t opA, int32_t opB, int64_t M, int64_t N, int64_t K, double alpha,
                                const void* A, int64_t lda, const void* B, int64_t ldb, double beta, const void* X,
                                int64_t ldx, double gamma, const void* Z, int64_t ldz, void* C, int64_t ldc,
                                int32_t flags) {
  try {
    g_static_err.clear();
    const int structure = flags & 31, cfg = (flags >> 8) & 0xff, nsplit = (flags >> 16) & 0xff;
    if (!zgemm_args_ok(opA, opB, M, N, K, A, lda, B, ldb, X, ldx, Z, ldz, C, ldc, flags)) return CHFSI_OK;
    if (nsplit > 1 && (double)nsplit * (double)M * (double)N * sizeof(zc) > (double)STATIC_SCRATCH_BYTES)
      throw Error(ST_EINVAL, "zgemm_static: the split-K partial tiles (" + std::to_string(nsplit) + " x " +
                                 std::to_string(M) + " x " + std::to_string(N) + " x 16 bytes) exceed the static " +
                                 "scratch of " + std::to_string(STATIC_SCRATCH_BYTES) + " bytes");
    void* P = static_scratch_ptr();
    GemmOp g;
    g.cfg = cfg;
    g.splitk = nsplit;
    g.opA = opA; g.opB = opB; g.M = M; g.N = N; g.K = K;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
    g.X = X; g.ldx = ldx; g.Z = Z; g.ldz = ldz;
    g.alpha = alpha; g.beta = beta; g.gamma = gamma;
    g.flags = structure;
    g.allow_splitk = true;
    zgemm(g, GemmWork{static_cast<zc*>(P), STATIC_SCRATCH_BYTES / sizeof(zc)}, (hipStream_t)stream);
    return CHFSI_OK;
  } catch (const Error& e) {
    g_static_err = e.what();
    (void)hipGetLastError();
    return (chfsi_status)e.code;
  } catch (const std::exception& e) {
    g_static_err = e.what();
    return CHFSI_EHIP;
  } catch (...) {
    g_static_err = "unknown error";
    return CHFSI_EHIP;
  }
}

chfsi_status chfsi_server_create(chfsi_server* out, const chfsi_server_config* cfg) {
  if (!out || !cfg) return CHFSI_EINVAL;
  *out = nullptr;
  if (cfg->workers < 1 || cfg->workers > 64 || cfg->hbm_budget_bytes <= 0) return CHFSI_EINVAL;
  chfsi_opts o = cfg->opts;
  if (o.degree < 1 || o.max_iter < 1 || o.lanczos_steps < 1 || o.lanczos_steps > JACOBI_LDS_MAX ||
      o.precision < 0 || o.precision > 3 || (o.qr_mode != 0 && o.qr_mode != 1))
    return CHFSI_EINVAL;
  chfsi_server s = new (std::nothrow) chfsi_server_s();
  if (!s) return CHFSI_ENOMEM;
  s->cfg = *cfg;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return CHFSI_EHIP;
  }
  for (int i = 0; i < cfg->workers; i++) {
    std::unique_ptr<Worker> w(new Worker());
    if (hipStreamCreateWithFlags(&w->st, hipStreamNonBlocking) != hipSuccess) {
      chfsi_server_destroy(s);
      return CHFSI_EHIP;
    }
    s->workers.push_back(std::move(w));
  }
  for (auto& w : s->workers) w->th = std::thread(server_worker, s, w.get());
  *out = s;
  return CHFSI_OK;
}

chfsi_status chfsi_server_submit(chfsi_server s, int64_t seq, int64_t n, const void* H, int64_t ldh, const void* S,
                                 int64_t lds, int64_t nev, int64_t nex, double tol, double* evals, void* X, int64_t ldx,
                                 int64_t* ticket) {
  if (!s || !ticket) return CHFSI_EINVAL;
  if (n < 1 || !block_sizes_ok(n, nev, nex) || !(tol > 0.0) || !H || !evals || ldh < n || (S && lds < n) ||
      (X && ldx < n))
    return CHFSI_EINVAL;
  std::unique_ptr<Req> r(new Req());
  r->seq = seq;
  r->n = n;
  r->nev = nev;
  r->nex = nex;
  r->H = (const zc*)H;
  r->ldh = ldh;
  r->S = (const zc*)S;
  r->lds = lds;
  r->tol = tol;
  r->evals = evals;
  r->X = (zc*)X;
  r->ldx = ldx;
  r->t_submit = std::chrono::steady_clock::now();
  std::lock_guard<std::mutex> lk(s->m);
  if (s->stop) return CHFSI_EINVAL;
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  if (!s->have_first) {
    s->t_first = r->t_submit;
    s->have_first = true;
  }
  s->submitted++;
  s->queue.push_back(r.get());
  s->reqs[r->ticket] = std::move(r);
  s->cv_work.notify_all();
  return CHFSI_OK;
}

chfsi_status chfsi_server_wait(chfsi_server s, int64_t ticket, chfsi_info* info, double* latency_seconds) {
  if (!s) return CHFSI_EINVAL;
  std::unique_lock<std::mutex> lk(s->m);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return CHFSI_EINVAL;
  Req* r = it->second.get();
  s->cv_done.wait(lk, [&] { return r->done; });
  if (info) *info = r->info;
  if (latency_seconds) *latency_seconds = std::chrono::duration<double>(r->t_end - r->t_submit).count();
  const chfsi_status st = (chfsi_status)r->status;
  if (st != CHFSI_OK) s->err = r->err;
  s->reqs.erase(it);
  return st;
}

chfsi_status chfsi_server_stats(chfsi_server s, chfsi_server_statistics* out) {
  if (!s || !out) return CHFSI_EINVAL;
  std::lock_guard<std::mutex> lk(s->m);
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->queued = (int64_t)s->queue.size();
  out->running = s->running;
  out->bytes_in_use = (int64_t)s->used;
  out->peak_bytes = (int64_t)s->peak;
  out->budget_bytes = s->cfg.hbm_budget_bytes;
  if (!s->lat.empty()) {
    std::vector<double> v = s->lat;
    std::sort(v.begin(), v.end());
    auto q = [&](double f) {
      const size_t i = (size_t)std::min<double>((double)v.size() - 1, std::ceil(f * v.size()) - 1);
      return v[i];
    };
    out->p50_latency = q(0.50);
    out->p99_latency = q(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_latency = sum / v.size();
    const double span = std::chrono::duration<double>(s->t_last - s->t_first).count();
    out->solves_per_second = span > 0 ? s->completed / span : 0.0;
  }
  return CHFSI_OK;
}

chfsi_status chfsi_server_release_sequence(chfsi_server s, int64_t seq) {
  if (!s) return CHFSI_EINVAL;
  std::lock_guard<std::mutex> lk(s->m);
  auto it = s->seqs.find(seq);
  if (it == s->seqs.end()) return CHFSI_OK;
  if (it->second->busy) return CHFSI_EINVAL;
  for (Req* r : s->queue)
    if (r->seq == seq) return CHFSI_EINVAL;
  s->used -= it->second->X.bytes;
  it->second->X.release();
  s->seqs.erase(it);
  for (auto& w : s->workers)
    if (w->factor_seq == seq) w->factor_seq = -1;  // a later sequence of this id brings its own S
  s->cv_work.notify_all();
  return CHFSI_OK;
}

const char* chfsi_server_last_error(chfsi_server s) { return s ? s->err.c_str() : "null server"; }

void chfsi_server_destroy(chfsi_server s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->stop = true;
    for (Req* r : s->queue) {
      r->status = CHFSI_EINVAL;
      r->err = "server destroyed before the request ran";
      r->done = true;
    }
    s->queue.clear();
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
  for (auto& w : s->workers)
    if (w->th.joinable()) w->th.join();
  for (auto& w : s->workers) {
    if (w->ctx) chfsi_release(w->ctx);
    if (w->st) (void)hipStreamDestroy(w->st);
  }
  for (auto& kv : s->seqs) kv.second->X.release();
  delete s;
}


// ---------------------------------------------------------------------------
// Batching
// ---------------------------------------------------------------------------
chfsi_status chfsi_batch_create(chfsi_batch* out, int32_t count, const int64_t* n, const chfsi_opts* opts,
                                int32_t use_graph) {
  if (!out) return CHFSI_EINVAL;
  *out = nullptr;
  if (count < 1 || count > 1024 || !n || (use_graph != 0 && use_graph != 1)) return CHFSI_EINVAL;
  for (int j = 0; j < count; j++)
    if (n[j] < 1) return CHFSI_EINVAL;
  chfsi_opts o;
  chfsi_default_opts(&o);
  if (opts) o = *opts;
  o.profile = 0;
  if (o.filter_tile != 0 && !zgemm_grouped_config_ok(o.filter_tile)) return CHFSI_EINVAL;
  // the grouped filter steps have FP64 and FP32 forms only
  if (o.precision == 3) return CHFSI_EINVAL;
  chfsi_batch b = new (std::nothrow) chfsi_batch_s();
  if (!b) return CHFSI_ENOMEM;
  try {
    CHFSI_HIP(hipGetDevice(&b->device));
    b->count = count;
    b->use_graph = use_graph != 0;
    b->opts = o;
    b->threads = std::min(count, 8);
    CHFSI_HIP(hipStreamCreateWithFlags(&b->gst, hipStreamNonBlocking));
    CHFSI_HIP(hipEventCreateWithFlags(&b->gdone, hipEventDisableTiming));
    for (int p = 0; p < 2; p++)
      for (int q = 0; q < 2; q++) CHFSI_HIP(hipEventCreate(&b->gt[p][q]));
    for (int j = 0; j < count; j++) {
      hipStream_t x = nullptr;
      CHFSI_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
      b->mst.push_back(x);
      hipEvent_t e = nullptr;
      CHFSI_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      b->ready.push_back(e);
      chfsi_ctx c = nullptr;
      const chfsi_status st = chfsi_create(&c, n[j], &o, x);
      if (st != CHFSI_OK) throw Error(st, "member context creation failed");
      b->mem.push_back(c);
    }
    const size_t m = (size_t)o.degree;
    for (int p = 0; p < 2; p++) {
      b->gp[p].ensure(m * count * sizeof(ZGemmParams));
      b->t0[p].ensure(m * (size_t)(count + 1) * sizeof(int64_t));
      b->ctr[p].ensure((size_t)8 * m * sizeof(int));
      b->e0[p].ensure(m * (size_t)(count + 1) * sizeof(int64_t));
      CHFSI_HIP(hipHostMalloc((void**)&b->he0[p], m * (size_t)(count + 1) * sizeof(int64_t), hipHostMallocDefault));
      CHFSI_HIP(hipHostMalloc((void**)&b->hgp[p], m * count * sizeof(ZGemmParams), hipHostMallocDefault));
      CHFSI_HIP(hipHostMalloc((void**)&b->ht0[p], m * (size_t)(count + 1) * sizeof(int64_t), hipHostMallocDefault));
    }
    if (o.filter_tile) b->cfg[0] = b->cfg[1] = o.filter_tile;
  } catch (const Error& e) {
    b->destroy();
    delete b;
    (void)hipGetLastError();
    return (chfsi_status)e.code;
  }
  *out = b;
  return CHFSI_OK;
}

chfsi_status chfsi_batch_solve(chfsi_batch b, const void* const* H, const int64_t* ldh, const void* const* S,
                               const int64_t* lds, const int64_t* nev, const int64_t* nex, double tol,
                               double* const* evals, void* const* X, const int64_t* ldx, chfsi_info* infos,
                               int32_t* statuses, chfsi_batch_report* report) {
  if (!b) return CHFSI_EINVAL;
  try {
    b->err.clear();
    batch_solve_impl(b, H, ldh, S, lds, nev, nex, tol, evals, X, ldx, infos, statuses, report);
    return CHFSI_OK;
  } catch (const Error& e) {
    b->err = e.what();
    (void)hipGetLastError();
    return (chfsi_status)e.code;
  } catch (const std::exception& e) {
    b->err = e.what();
    return CHFSI_EHIP;
  }
}

chfsi_status chfsi_batch_reset(chfsi_batch b) {
  if (!b) return CHFSI_EINVAL;
  for (auto c : b->mem) c->warm_valid = false;
  return CHFSI_OK;
}

const char* chfsi_batch_last_error(chfsi_batch b) { return b ? b->err.c_str() : "null batch"; }

void chfsi_batch_release(chfsi_batch b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  b->destroy();
  delete b;
}

}  // extern "C"
