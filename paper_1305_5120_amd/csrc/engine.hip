// Solver engine and C ABI of the ChFSI library.
//
// Host-side orchestration of Algorithm 1 (arXiv 1305.5120): every numerical
// step runs in this library's kernels (zgemm.hip, kernels.hip) on the
// context's stream; the host only sequences launches, reads back the k_a Ritz
// values and residual norms once per outer iteration and takes the locking
// decision.
#include <chrono>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/chfsi.h"
#include "gemm.hpp"
#include "kernels.hpp"

using namespace chfsi;

namespace {

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

}  // namespace

struct chfsi_ctx_s {
  int64_t n = 0;
  chfsi_opts opts{};
  hipStream_t st = nullptr;
  std::string err;

  // n x n: standard form, Cholesky factor, its inverse, work; FP32 copy of A
  DBuf A, L, Linv, W, A32;
  // FP32 filter blocks (mixed precision)
  DBuf Y32, Y32b;
  bool have_factors = false;
  // n x k blocks
  DBuf Y, Yb, F, Qb, Wk, Wz;
  int64_t kcap = 0;
  // k x k and small
  DBuf G, Z, Z2, G2, Ztmp, mu, rho, rank, norms, flags;
  DBuf P;  // split-K partial tiles
  size_t P_elems = 0;
  // Householder
  DBuf hpart, htop, tau, Tall, gram, Vp, Wt, W2;
  // Lanczos
  DBuf LV, Lw, Lh, Lab, mvpart, Tsm, Tz, Tz2, Tw, npart;
  // host staging (pinned)
  double* hbuf = nullptr;
  size_t hbuf_elems = 0;

  // warm state (Y holds the block)
  bool warm_valid = false;
  int64_t warm_k = 0;
  double warm_a0 = 0, warm_a = 0;

  // filter timing and work, per precision (0 FP64, 1 FP32)
  std::vector<EventPair> fev;
  double filt_kernel_s[2] = {0, 0};
  int filt_launches[2] = {0, 0};
  double filt_flops[2] = {0, 0};
  int last_filter_prec = 0;
  void reset_filter_stats() {
    for (int i = 0; i < 2; i++) {
      filt_kernel_s[i] = 0;
      filt_launches[i] = 0;
      filt_flops[i] = 0;
    }
  }

  GemmWork gw() const { return GemmWork{P.z(), P_elems}; }

  void ensure_host(size_t elems) {
    if (hbuf_elems >= elems) return;
    if (hbuf) (void)hipHostFree(hbuf);
    hbuf = nullptr;
    hbuf_elems = 0;
    CHFSI_HIP(hipHostMalloc((void**)&hbuf, elems * sizeof(double), hipHostMallocDefault));
    hbuf_elems = elems;
  }

  void ensure_nn() {
    const size_t b = (size_t)n * n * sizeof(zc);
    A.ensure(b);
    L.ensure(b);
    Linv.ensure(b);
    W.ensure(b);
  }

  void ensure_k(int64_t k) {
    if (k <= kcap && Y.p) return;
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
    mu.release(); mu.ensure((size_t)kk * sizeof(double));
    rho.release(); rho.ensure((size_t)kk * sizeof(double));
    rank.release(); rank.ensure((size_t)kk * sizeof(int));
    P_elems = 8 * (size_t)kk * kk + (size_t)std::max(4, opts.filter_splitk) * n * kk + ((size_t)1 << 16);
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
  }

  void ensure_small() {
    norms.ensure(8 * sizeof(double));
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
    for (DBuf* b : {&A32, &Y32, &Y32b, &A, &L, &Linv, &W, &Y, &Yb, &F, &Qb, &Wk, &Wz, &G, &Z, &Z2, &G2, &Ztmp, &mu, &rho, &rank, &norms,
                    &flags, &P, &hpart, &htop, &tau, &Tall, &gram, &Vp, &Wt, &W2, &LV, &Lw, &Lh, &Lab, &mvpart, &Tsm,
                    &Tz, &Tz2, &Tw, &npart})
      b->release();
    if (hbuf) (void)hipHostFree(hbuf);
    hbuf = nullptr;
    for (auto& e : fev) {
      if (e.a) (void)hipEventDestroy(e.a);
      if (e.b) (void)hipEventDestroy(e.b);
    }
    fev.clear();
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
  int chol_factor(int64_t m, const zc* src, int64_t lds, zc* Wb, zc* Lb, zc* Lib, int64_t ld) {
    const int64_t NB = CHOL_NB;
    copy2d(src, lds, Wb, ld, m, m, st);
    fill_i32(flags.i(), 1, INT_MAX, st);
    for (int64_t j0 = 0; j0 < m; j0 += NB) {
      const int64_t nb = std::min(NB, m - j0), r = m - j0 - nb;
      chol_diag(Wb, ld, Lb, ld, Lib, ld, j0, nb, flags.i(), st);
      if (r > 0) {
        // L21 = W21 L11^{-H}
        gemm(OP_N, OP_C, r, nb, nb, 1.0, Wb + (j0 + nb) + j0 * ld, ld, Lib + j0 + j0 * ld, ld, Lb + (j0 + nb) + j0 * ld,
             ld, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_TRI_B_UPPER, false);
        // W22 -= L21 L21^H (lower tiles)
        zc* W22 = Wb + (j0 + nb) + (j0 + nb) * ld;
        const zc* L21 = Lb + (j0 + nb) + j0 * ld;
        gemm(OP_N, OP_C, r, r, nb, -1.0, L21, ld, L21, ld, W22, ld, 1.0, W22, ld, 0.0, nullptr, 0, GEMM_OUT_LOWER, false);
      }
    }
    zero_strict_upper(Lb, ld, m, st);
    CHFSI_HIP(hipMemcpyAsync(hbuf, flags.p, sizeof(int), hipMemcpyDeviceToHost, st));
    sync();
    int info;
    std::memcpy(&info, hbuf, sizeof(int));
    if (info != INT_MAX) return info;
    // Lib: off-diagonal blocks by recursive doubling,
    //   inv([[L11, 0], [L21, L22]]) = [[X11, 0], [-X22 L21 X11, X22]]
    for (int64_t s = NB; s < m; s *= 2) {
      for (int64_t i0 = 0; i0 + s < m; i0 += 2 * s) {
        const int64_t b = std::min(s, m - i0 - s);
        const zc* L21 = Lb + (i0 + s) + i0 * ld;
        const zc* X11 = Lib + i0 + i0 * ld;
        const zc* X22 = Lib + (i0 + s) + (i0 + s) * ld;
        zc* T = Wb;
        gemm(OP_N, OP_N, b, s, s, 1.0, L21, ld, X11, ld, T, ld, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_TRI_B_LOWER);
        gemm(OP_N, OP_N, b, s, b, -1.0, X22, ld, T, ld, Lib + (i0 + s) + i0 * ld, ld, 0.0, nullptr, 0, 0.0, nullptr, 0,
             GEMM_TRI_A_LOWER);
      }
    }
    zero_strict_upper(Lib, ld, m, st);
    return 0;
  }

  void cholesky(const zc* S, int64_t lds) {
    const int info = chol_factor(n, S, lds, W.z(), L.z(), Linv.z(), n);
    if (info) {
      have_factors = false;
      throw Error(ST_ENOTPD, "S is not positive definite: pivot of column " + std::to_string(info - 1) + " is not positive");
    }
    have_factors = true;
  }

  void reduce(const zc* H, int64_t ldh, const zc* S, int64_t lds) {
    ensure_nn();
    ensure_small();
    if (S) cholesky(S, lds);
    else if (!have_factors) throw Error(ST_EINVAL, "no cached factor of S: pass S");
    // A = Linv H Linv^H
    gemm(OP_N, OP_N, n, n, n, 1.0, Linv.z(), n, H, ldh, W.z(), n, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_TRI_A_LOWER);
    gemm(OP_N, OP_C, n, n, n, 1.0, W.z(), n, Linv.z(), n, A.z(), n, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_TRI_B_UPPER);
    hermitize(A.z(), n, n, st);
  }

  // ------------------------------------------------------------------------
  // Hermitian eigensolver (Jacobi) into w (device, ascending), Zo (device)
  // ------------------------------------------------------------------------
  void eigh(const zc* Gp, int64_t ldg, int64_t k, double* w, zc* Zo, int64_t ldz) {
    if (k <= JACOBI_LDS_MAX) {
      jacobi_small(Gp, ldg, k, w, Zo, ldz, Ztmp.z(), nullptr, st);
      return;
    }
    zc *g0 = G2.z(), *z0 = Ztmp.z(), *g1 = Z2.z();
    // Z2 and a second k x k buffer: reuse Wz's storage for the Z ping-pong
    zc* z1 = Wz.z();
    jacobi_init(Gp, ldg, k, g0, z0, st);
    double* nr = norms.d();
    jacobi_norms(g0, k, npart.d(), nr, st);  // nr[0] = off, nr[1] = all (fro2)
    CHFSI_HIP(hipMemcpyAsync(hbuf, nr, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
    const double fro2 = hbuf[1];
    double off2 = hbuf[0];
    const int64_t K2 = k + (k & 1);
    for (int sweep = 0; sweep < 100 && off2 > 1e-32 * fro2 && off2 != 0.0; sweep++) {
      fill_i32(flags.i() + 1, 1, 0, st);
      for (int64_t r = 0; r < K2 - 1; r++) {
        jacobi_round(g0, g1, z0, z1, k, r, nr + 1, flags.i() + 1, st);
        std::swap(g0, g1);
        std::swap(z0, z1);
      }
      jacobi_norms(g0, k, npart.d(), nr + 2, st);
      CHFSI_HIP(hipMemcpyAsync(hbuf, nr + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      CHFSI_HIP(hipMemcpyAsync(hbuf + 2, flags.i() + 1, sizeof(int), hipMemcpyDeviceToHost, st));
      sync();
      off2 = hbuf[0];
      int rot;
      std::memcpy(&rot, hbuf + 2, sizeof(int));
      if (!rot) break;
    }
    jacobi_sort(g0, z0, k, w, rank.i(), Zo, ldz, st);
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
  // One CholeskyQR pass: G = Yin^H Yin = Lg Lg^H, Qo = Yin Lg^{-H}.  False
  // when the Gram matrix is not numerically positive definite.
  // ------------------------------------------------------------------------
  bool cholqr_pass(const zc* Yin, int64_t ldy, int64_t k, zc* Qo, int64_t ldq) {
    gemm(OP_C, OP_N, k, k, n, 1.0, Yin, ldy, Yin, ldy, G.z(), k);
    hermitize(G.z(), k, k, st);
    if (chol_factor(k, G.z(), k, G2.z(), Z2.z(), Ztmp.z(), k) != 0) return false;
    gemm(OP_N, OP_C, n, k, k, 1.0, Yin, ldy, Ztmp.z(), k, Qo, ldq, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_TRI_B_UPPER);
    return true;
  }

  // Orthonormal basis of span(F) (F: n x k, ld n, destroyed) into Qo.
  // CholeskyQR2 (two passes; orthogonal to working precision while
  // cond(F) is below ~1e7); if a Gram matrix is not positive definite the
  // block is too ill-conditioned for it and Householder QR takes over on
  // the best basis at hand.  Returns true when Householder was used.
  bool orthonormalize(zc* Fp, int64_t k, zc* Qo, int64_t ldq) {
    if (opts.qr_mode == 0) {
      zc* mid = Wk.z();
      if (cholqr_pass(Fp, n, k, mid, n)) {
        if (cholqr_pass(mid, n, k, Qo, ldq)) return false;
        qr(mid, n, k, Qo, ldq);
        return true;
      }
    }
    qr(Fp, n, k, Qo, ldq);
    return true;
  }

  // ------------------------------------------------------------------------
  // Chebyshev filter on Y (n x ka); Yb same shape as work.  Returns the
  // buffer holding the result (Y or Yb).
  // ------------------------------------------------------------------------
  zc* filter(const zc* Ap, int64_t lda, zc* Yp, int64_t ldy, zc* Ybp, int64_t ldyb, int64_t ka, int m, double a, double b,
             double a0) {
    return static_cast<zc*>(filter_any(PREC_F64, Ap, lda, Yp, ldy, Ybp, ldyb, ka, m, a, b, a0));
  }

  // The filter in either precision: element type zc (FP64) or cc (FP32).
  void* filter_any(int prec, const void* Ap, int64_t lda, void* Yp, int64_t ldy, void* Ybp, int64_t ldyb, int64_t ka, int m,
                   double a, double b, double a0) {
    const double e = (b - a) / 2.0, c = (b + a) / 2.0;
    const double sigma1 = e / (a0 - c);
    const double tau_ = 2.0 / sigma1;
    const bool prof = opts.profile != 0;
    if (prof && (int)fev.size() < m) {
      for (int i = (int)fev.size(); i < m; i++) {
        EventPair ep;
        CHFSI_HIP(hipEventCreate(&ep.a));
        CHFSI_HIP(hipEventCreate(&ep.b));
        fev.push_back(ep);
      }
    }
    auto step = [&](int i, const void* cur, int64_t ldc, void* out, int64_t ldo, double al, double be, double ga,
                    const void* prev, int64_t ldp) {
      if (prof) CHFSI_HIP(hipEventRecord(fev[i].a, st));
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
      if (prof) CHFSI_HIP(hipEventRecord(fev[i].b, st));
    };
    // Y_1 = (sigma1/e)(A - cI) Y_0
    const double al1 = sigma1 / e;
    step(0, Yp, ldy, Ybp, ldyb, al1, -al1 * c, 0.0, nullptr, 0);
    void *cur = Ybp, *prev = Yp;
    int64_t ldc = ldyb, ldp = ldy;
    double sigma = sigma1;
    for (int i = 2; i <= m; i++) {
      const double sn = 1.0 / (tau_ - sigma);
      const double al = 2.0 * sn / e;
      // Y_i = al (A - cI) Y_{i-1} - sigma sn Y_{i-2}, written over Y_{i-2}
      step(i - 1, cur, ldc, prev, ldp, al, -al * c, -sigma * sn, prev, ldp);
      std::swap(cur, prev);
      std::swap(ldc, ldp);
      sigma = sn;
    }
    filt_launches[prec] += m;
    filt_flops[prec] += 8.0 * (double)n * (double)n * (double)ka * (double)m;
    last_filter_prec = prec;
    return cur;
  }

  void collect_filter_events(int m) {
    if (!opts.profile) return;
    for (int i = 0; i < m && i < (int)fev.size(); i++) {
      float ms = 0.f;
      CHFSI_HIP(hipEventElapsedTime(&ms, fev[i].a, fev[i].b));
      filt_kernel_s[last_filter_prec] += ms * 1e-3;
    }
  }

  // ------------------------------------------------------------------------
  // Rayleigh-Ritz on Qa (n x ka, orthonormal) -> Yo = Qa Z, mu (device),
  // WZo = A Yo (through W Z).
  // ------------------------------------------------------------------------
  void rayleigh_ritz(const zc* Ap, int64_t lda, const zc* Qa, int64_t ldq, int64_t ka, zc* Yo, int64_t ldyo, double* mu_d,
                     zc* Wbuf, zc* WZo) {
    gemm(OP_N, OP_N, n, ka, n, 1.0, Ap, lda, Qa, ldq, Wbuf, n);
    gemm(OP_C, OP_N, ka, ka, n, 1.0, Qa, ldq, Wbuf, n, G.z(), ka);
    hermitize(G.z(), ka, ka, st);
    eigh(G.z(), ka, ka, mu_d, Z.z(), ka);
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

// Run the whole of Algorithm 1.
void solve_impl(chfsi_ctx c, const zc* H, int64_t ldh, const zc* S, int64_t lds, int64_t nev, int64_t nex, const zc* Vw,
                int64_t ldv, int64_t kw, double tol, double* evals, zc* X, int64_t ldx, chfsi_info* info) {
  const int64_t n = c->n;
  const int64_t k = nev + nex;
  if (nev < 1 || nex < 0 || k > n) throw Error(ST_EINVAL, "need 1 <= nev and nev + nex <= n");
  if (!(tol > 0.0)) throw Error(ST_EINVAL, "tol must be positive");
  if (kw < 0 || kw > k) throw Error(ST_EINVAL, "kw out of range");
  check_ptr(H, "H");
  check_ld(ldh, n, "ldh");
  if (S) check_ld(lds, n, "lds");
  if (Vw && kw > 0) check_ld(ldv, n, "ldv");
  if (X) check_ld(ldx, n, "ldx");
  check_ptr(evals, "evals");
  const chfsi_opts& o = c->opts;
  hipStream_t st = c->st;

  chfsi_info inf{};
  auto t_start = std::chrono::steady_clock::now();
  auto now = [&]() { return std::chrono::steady_clock::now(); };
  auto secs = [](std::chrono::steady_clock::time_point a, std::chrono::steady_clock::time_point b) {
    return std::chrono::duration<double>(b - a).count();
  };
  c->reset_filter_stats();

  c->ensure_nn();
  c->ensure_small();
  const bool state_ok = c->warm_valid && c->warm_k == k && c->Y.p;
  c->ensure_k(k);
  // a warm block meant for a changed S goes through the generalized space:
  // X_old = L_old^{-H} Y (into F) before the new factor replaces L_old
  const bool use_state = (Vw == nullptr || kw == 0) && state_ok;
  if (use_state && S && c->have_factors)
    c->gemm(OP_C, OP_N, n, k, n, 1.0, c->Linv.z(), n, c->Y.z(), n, c->F.z(), n, 0.0, nullptr, 0, 0.0, nullptr, 0,
            GEMM_TRI_A_UPPER);

  auto t0 = now();
  c->reduce(H, ldh, S, lds);
  const bool mixed = o.precision == 1;
  if (mixed) {
    c->A32.ensure((size_t)n * n * sizeof(cc));
    c->Y32.ensure((size_t)n * k * sizeof(cc));
    c->Y32b.ensure((size_t)n * k * sizeof(cc));
    to_f32(c->A.z(), n, (cc*)c->A32.p, n, n, n, st);
  }
  c->sync();
  inf.t_reduce = secs(t0, now());

  t0 = now();
  double lz[3];
  c->lanczos(c->A.z(), n, o.lanczos_steps, o.seed, 1u, lz);
  inf.theta_min = lz[0];
  inf.b_upper = lz[2];
  c->lanczos(H, ldh, o.lanczos_steps, o.seed, 2u, lz);
  inf.h_H = std::max(std::fabs(lz[0]), std::fabs(lz[1]));
  inf.t_lanczos = secs(t0, now());

  zc* Y = c->Y.z();
  zc* Yb = c->Yb.z();
  zc* F = c->F.z();
  zc* Qb = c->Qb.z();
  zc* Wk = c->Wk.z();
  zc* Wz = c->Wz.z();
  double* mu_d = c->mu.d();
  double* rho_d = c->rho.d();
  double* hb = c->hbuf;

  // start block
  bool warm = false;
  if (Vw && kw > 0) {
    c->gemm(OP_C, OP_N, n, kw, n, 1.0, c->L.z(), n, Vw, ldv, Y, n, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_TRI_A_UPPER);
    if (kw < k) random_block(o.seed, 3u, n, k - kw, kw, Y + kw * n, n, st);
    warm = true;
  } else if (use_state) {
    if (S) c->gemm(OP_C, OP_N, n, k, n, 1.0, c->L.z(), n, F, n, Y, n, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_TRI_A_UPPER);
    warm = true;
  } else {
    random_block(o.seed, 3u, n, k, 0, Y, n, st);
  }
  copy2d(Y, n, F, n, n, k, st);
  inf.qr_householder += c->orthonormalize(F, k, Qb, n) ? 1 : 0;
  double a0, a;
  const double b = inf.b_upper;
  if (warm && c->warm_valid && c->warm_k == k) {
    copy2d(Qb, n, Y, n, n, k, st);
    a0 = c->warm_a0;
    a = c->warm_a;
  } else {
    c->rayleigh_ritz(c->A.z(), n, Qb, n, k, Y, n, mu_d, Wk, nullptr);
    CHFSI_HIP(hipMemcpyAsync(hb, mu_d, k * sizeof(double), hipMemcpyDeviceToHost, st));
    c->sync();
    a0 = std::min(inf.theta_min, hb[0]);
    a = hb[k - 1];
  }
  inf.warm_start = warm ? 1 : 0;
  c->warm_valid = false;  // the block is being rewritten

  std::vector<double> lam(k, NAN), rho_lock(k, 0.0);
  int64_t cl = 0;
  int it = 0;
  const double hs = tol * inf.h_H;
  bool converged = false;
  std::vector<hipEvent_t> ev(5);
  for (auto& e : ev) CHFSI_HIP(hipEventCreate(&e));
  struct EvGuard {
    std::vector<hipEvent_t>& v;
    ~EvGuard() {
      for (auto e : v) (void)hipEventDestroy(e);
    }
  } evg{ev};
  // Mixed precision: the filter runs in complex FP32 while the first active
  // column's generalized residual is above MIXED_SWITCH * h_H and still
  // falling at least twofold per FP32 iteration; that column then gets FP64
  // filtering until it locks.  Everything else stays FP64, and locking uses
  // the FP64 residuals, so the accepted pairs meet the same tolerance.
  const double MIXED_SWITCH = 1e-5;
  int64_t fp64_col = -1, prev_col = -1;
  double prev_rho = INFINITY;
  bool prev32 = false;
  for (it = 1; it <= o.max_iter; it++) {
    const int64_t ka = k - cl;
    bool use32 = false;
    if (mixed) {
      use32 = fp64_col != cl;
      if (use32 && prev_col == cl && prev_rho <= MIXED_SWITCH * inf.h_H) {
        use32 = false;
        fp64_col = cl;
      }
    }
    CHFSI_HIP(hipEventRecord(ev[0], st));
    if (use32) {
      cc* y32 = (cc*)c->Y32.p;
      cc* y32b = (cc*)c->Y32b.p;
      to_f32(Y + cl * n, n, y32, n, n, ka, st);
      void* r32 = c->filter_any(PREC_F32, c->A32.p, n, y32, n, y32b, n, ka, o.degree, a, b, a0);
      to_f64((const cc*)r32, n, F + cl * n, n, n, ka, st);
      inf.iterations_fp32++;
    } else {
      zc* res = c->filter(c->A.z(), n, Y + cl * n, n, Yb + cl * n, n, ka, o.degree, a, b, a0);
      copy2d(res, n, F + cl * n, n, n, ka, st);
    }
    CHFSI_HIP(hipEventRecord(ev[1], st));
    if (cl > 0) copy2d(Y, n, F, n, n, cl, st);
    inf.qr_householder += c->orthonormalize(F, k, Qb, n) ? 1 : 0;
    CHFSI_HIP(hipEventRecord(ev[2], st));
    c->rayleigh_ritz(c->A.z(), n, Qb + cl * n, n, ka, Y + cl * n, n, mu_d, Wk, Wz);
    CHFSI_HIP(hipEventRecord(ev[3], st));
    c->residual_norms(c->L.z(), n, Wz, Y + cl * n, n, ka, mu_d, Wk, F, rho_d);
    CHFSI_HIP(hipMemcpyAsync(hb, mu_d, ka * sizeof(double), hipMemcpyDeviceToHost, st));
    CHFSI_HIP(hipMemcpyAsync(hb + ka, rho_d, ka * sizeof(double), hipMemcpyDeviceToHost, st));
    CHFSI_HIP(hipEventRecord(ev[4], st));
    c->sync();
    float ms[4];
    for (int i = 0; i < 4; i++) CHFSI_HIP(hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]));
    inf.t_filter += ms[0] * 1e-3;
    inf.t_qr += ms[1] * 1e-3;
    inf.t_rr += ms[2] * 1e-3;
    inf.t_resid += ms[3] * 1e-3;
    c->collect_filter_events(o.degree);
    const double* mu = hb;
    const double* rho = hb + ka;
    for (int64_t j = 0; j < ka; j++)
      if (!std::isfinite(mu[j]) || !std::isfinite(rho[j]))
        throw Error(ST_ENAN, "non-finite Ritz value or residual at iteration " + std::to_string(it));
    int64_t nl = 0;
    while (cl + nl < nev && nl < ka && rho[nl] <= hs) {
      lam[cl + nl] = mu[nl];
      rho_lock[cl + nl] = rho[nl];
      nl++;
    }
    for (int64_t j = nl; j < ka; j++) {
      lam[cl + j] = mu[j];
      rho_lock[cl + j] = rho[j];
    }
    if (mixed) {
      // stall of an FP32 iteration on the same first column
      if (prev32 && prev_col == cl && rho[0] > 0.5 * prev_rho) fp64_col = cl;
      prev32 = use32;
      prev_col = cl + nl;
      prev_rho = nl < ka ? rho[nl] : INFINITY;
    }
    cl += nl;
    a = mu[ka - 1];
    a0 = std::min(a0, mu[0]);
    inf.converged = (int32_t)cl;
    if (cl >= nev) {
      converged = true;
      break;
    }
  }
  inf.iterations = std::min(it, o.max_iter);
  inf.a0 = a0;
  inf.a = a;
  const int64_t nout = converged ? nev : cl;
  double mx = 0.0;
  for (int64_t j = 0; j < nev; j++) {
    evals[j] = j < nout ? lam[j] : NAN;
    if (j < nout) mx = std::max(mx, rho_lock[j] / inf.h_H);
  }
  inf.max_rel_residual = mx;
  if (X && nev > 0)
    c->gemm(OP_C, OP_N, n, nev, n, 1.0, c->Linv.z(), n, Y, n, X, ldx, 0.0, nullptr, 0, 0.0, nullptr, 0, GEMM_TRI_A_UPPER);
  c->sync();
  // warm state for the next problem of the sequence
  c->warm_valid = true;
  c->warm_k = k;
  c->warm_a0 = a0;
  c->warm_a = a;
  inf.filter_flops = c->filt_flops[0] + c->filt_flops[1];
  inf.filter_launches = c->filt_launches[0] + c->filt_launches[1];
  inf.filter_kernel_seconds = c->filt_kernel_s[0] + c->filt_kernel_s[1];
  inf.filter_flops_fp32 = c->filt_flops[1];
  inf.filter_launches_fp32 = c->filt_launches[1];
  inf.filter_kernel_seconds_fp32 = c->filt_kernel_s[1];
  inf.t_total = secs(t_start, now());
  if (info) *info = inf;
  if (!converged)
    throw Error(ST_ENOCONV, "not converged after " + std::to_string(o.max_iter) + " iterations (" + std::to_string(cl) +
                                " of " + std::to_string(nev) + " locked)");
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
  if (o.degree < 1 || o.max_iter < 1 || o.lanczos_steps < 1 || o.lanczos_steps > JACOBI_LDS_MAX || (o.precision != 0 && o.precision != 1) ||
      (o.qr_mode != 0 && o.qr_mode != 1) || o.filter_tile < 0 || o.filter_tile >= zgemm_num_configs() ||
      o.filter_splitk < 0 || o.filter_splitk > 16)
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

const char* chfsi_last_error(chfsi_ctx c) { return c ? c->err.c_str() : "null context"; }

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
    const int64_t n = c->n;
    if (c->opts.precision == 1) {
      // mixed precision: the filter itself in complex FP32
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
    c->collect_filter_events(m);
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
    if (M < 0 || N < 0 || K < 0 || (opA != 0 && opA != 1) || (opB != 0 && opB != 1) || (flags & 0xff0000e0) ||
        cfg >= zgemm_num_configs())
      throw Error(ST_EINVAL, "zgemm: bad sizes, ops or flags");
    if (M == 0 || N == 0) return;
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
    c->ensure_small();
    // split-K scratch: the requested split, or 16-way for small outputs
    size_t need = (cdiv(M, 32) * cdiv(N, 32) < 256) ? (size_t)M * N * 16 : 0;
    if (nsplit > 1) need = std::max(need, (size_t)M * N * nsplit);
    if (need && c->P_elems < need) {
      c->P.release();
      c->P.ensure(need * sizeof(zc));
      c->P_elems = need;
    }
    c->gemm(opA, opB, M, N, K, alpha, (const zc*)A, lda, (const zc*)B, ldb, (zc*)C, ldc, beta, (const zc*)X, ldx, gamma,
            (const zc*)Z, ldz, structure, !(structure & GEMM_OUT_LOWER), false, cfg, nsplit);
    c->sync();
  });
}

}  // extern "C"
