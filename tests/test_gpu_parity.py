"""Parity of the gfx950 library (through its C ABI) with the CPU oracle.

Every step of Algorithm 1 is compared element by element with the oracle on
the same seeded inputs, at sizes that span several tiles and leave ragged
tails; the whole solve is compared on the n=512 configuration and on a short
warm-started sequence.  Tolerances (FP64 throughout):
  * single dense steps (filter, products, QR, reduction): relative Frobenius
    error <= 1e-12 (the two sides sum in different orders; cond(L) ~ 1);
  * eigenvalues: |dlam| <= 1e-10 |lam| or <= 1e-12 ||H||_2;
  * residuals: ||H x - lam S x|| <= 1e-10 ||H||_2 (the paper's tolerance).
"""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle
import workloads
from tests import _checks

pytestmark = pytest.mark.gpu


def _t(a):
    """numpy matrix -> column-major complex128 device tensor of the same shape."""
    import torch
    a = np.asarray(a, dtype=np.complex128)
    return torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda").mT


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _rng(s):
    return np.random.default_rng(s)


def _cg(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# --------------------------------------------------------------------------
# generator
# --------------------------------------------------------------------------

def test_philox_known_answers_bit_exact(lib):
    import os
    rows = [l.split() for l in open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    v = np.array([[int(x, 16) for x in r] for r in rows], dtype=np.uint64)
    ctx = lib.create(8)
    out = lib.philox(ctx, v[:, 0:4].astype(np.uint32), v[:, 4:6].astype(np.uint32))
    assert np.array_equal(out, v[:, 6:10].astype(np.uint32))
    # and the oracle's generator on a batch of counters
    rng = _rng(1)
    ctr = rng.integers(0, 2**32, size=(64, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(64, 2), dtype=np.uint64).astype(np.uint32)
    out = lib.philox(ctx, ctr, key)
    for i in range(64):
        assert np.array_equal(out[i], oracle.philox4x32_10(ctr[i], key[i]))


def test_random_block_matches_oracle(lib):
    n, k = 333, 7
    ctx = lib.create(n)
    Y = _np(lib.random_block(ctx, 12345, 3, k, col0=5))
    ref = oracle.gauss_block(12345, 3, n, k, col0=5)
    # same Philox bits; log / sin / cos may differ in the last bit
    assert np.abs(Y - ref).max() <= 1e-14 * np.abs(ref).max()


# --------------------------------------------------------------------------
# dense products (the filter's kernel in all its modes)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("opA,opB", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("M,N,K", [(77, 45, 131), (200, 130, 70), (20, 20, 3000), (1, 1, 1)])
def test_zgemm_against_definition(lib, opA, opB, M, N, K):
    rng = _rng(M + N + K + opA * 2 + opB)
    A = _cg(rng, (M, K) if opA == 0 else (K, M))
    B = _cg(rng, (K, N) if opB == 0 else (N, K))
    X = _cg(rng, (M, N))
    Z = _cg(rng, (M, N))
    ctx = lib.create(8)
    C = lib.zgemm(ctx, opA, opB, _t(A), _t(B), alpha=0.7, beta=-0.3, X=_t(X), gamma=1.9, Z=_t(Z))
    opa = A if opA == 0 else A.conj().T
    opb = B if opB == 0 else B.conj().T
    ref = 0.7 * (opa @ opb) - 0.3 * X + 1.9 * Z
    assert _rel(_np(C), ref) <= 1e-13


@pytest.mark.parametrize("opA,opB", [(0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("split", [1, 4])
def test_zgemm_eight_wave_tile_with_conjugate_operands(lib, opA, opB, split):
    """The eight-wave 64 x 64 tile (configuration 11) with conjugate-
    transposed operands and the three-term epilogue, ragged over several
    tiles, with and without a K split."""
    rng = _rng(1400 + 2 * opA + opB + split)
    M, N, K = 333, 141, 500
    A = _cg(rng, (M, K) if opA == 0 else (K, M))
    B = _cg(rng, (K, N) if opB == 0 else (N, K))
    X, Z = _cg(rng, (M, N)), _cg(rng, (M, N))
    ctx = lib.create(8)
    C = _np(lib.zgemm(ctx, opA, opB, _t(A), _t(B), alpha=0.7, beta=-0.3, X=_t(X), gamma=1.9, Z=_t(Z),
                      flags=(11 << 8) | (split << 16)))
    opa = A if opA == 0 else A.conj().T
    opb = B if opB == 0 else B.conj().T
    ref = 0.7 * (opa @ opb) - 0.3 * X + 1.9 * Z
    assert np.abs(C - ref).max() <= 1e-13 * np.abs(ref).max()


def test_zgemm_triangular_structure_flags(lib):
    rng = _rng(9)
    n = 150
    Lm = np.tril(_cg(rng, (n, n)))
    B = _cg(rng, (n, 40))
    ctx = lib.create(8)
    for opA, flag, opa in ((0, 1, Lm), (1, 2, Lm.conj().T)):
        C = lib.zgemm(ctx, opA, 0, _t(Lm), _t(B), flags=flag)
        assert _rel(_np(C), opa @ B) <= 1e-13
    Bl = np.tril(_cg(rng, (n, n)))
    Am = _cg(rng, (60, n))
    C = lib.zgemm(ctx, 0, 0, _t(Am), _t(Bl), flags=4)
    assert _rel(_np(C), Am @ Bl) <= 1e-13
    C = lib.zgemm(ctx, 0, 1, _t(Am), _t(Bl), flags=8)
    assert _rel(_np(C), Am @ Bl.conj().T) <= 1e-13


@pytest.mark.parametrize("flag", [1, 2, 16, 8 | 16])
@pytest.mark.parametrize("tile,split", [(0, 0), (1, 4), (7, 1), (2, 8), (11, 1), (11, 4)])
def test_zgemm_structured_products_many_tile_rows(lib, flag, tile, split):
    """Triangular op(A) (lower, upper), lower-only output, and upper op(B)
    with lower-only output over 18 tile rows (an odd count: the products
    deal their rows heaviest / lightest alternately), several column tiles,
    automatic and explicit tiles and K splits."""
    rng = _rng(100 + flag)
    n, w = 1100, 300
    ctx = lib.create(8)
    bits = flag | (tile << 8) | (split << 16)
    if flag in (1, 2):
        Am = np.tril(_cg(rng, (n, n))) if flag == 1 else np.triu(_cg(rng, (n, n)))
        B = _cg(rng, (n, w))
        C = lib.zgemm(ctx, 0, 0, _t(Am), _t(B), flags=bits)
        assert _rel(_np(C), Am @ B) <= 1e-13
    elif flag == 16:
        Am = _cg(rng, (n, 500))
        B = _cg(rng, (500, n))
        C = _np(lib.zgemm(ctx, 0, 0, _t(Am), _t(B), flags=bits))
        ref = Am @ B
        low = np.tril_indices(n)
        assert np.linalg.norm(C[low] - ref[low]) <= 1e-13 * np.linalg.norm(ref[low])
    else:
        Am = _cg(rng, (n, n))
        Bl = np.tril(_cg(rng, (n, n)))
        C = _np(lib.zgemm(ctx, 0, 1, _t(Am), _t(Bl), flags=bits))
        ref = Am @ Bl.conj().T
        low = np.tril_indices(n)
        assert np.linalg.norm(C[low] - ref[low]) <= 1e-13 * np.linalg.norm(ref[low])


@pytest.mark.parametrize("flag,split", [(0, 1), (0, 4), (1, 4), (2, 8), (16, 1)])
def test_zgemm_eight_wave_tile(lib, flag, split):
    """The 64 x 64 tile with eight waves (configuration 11) in the general
    product: plain, lower- and upper-triangular op(A) with K splits, and the
    lower-triangle output, with the three-term epilogue; ragged sizes over
    several tiles."""
    rng = _rng(1100 + flag + split)
    if flag in (1, 2):  # square triangular op(A)
        M = K = 1100
        N = 141
    else:
        M, K = 333, 500
        N = M if flag == 16 else 141
    Am = _cg(rng, (M, K))
    if flag == 1:
        Am = np.tril(Am)
    elif flag == 2:
        Am = np.triu(Am)
    B = _cg(rng, (K, N))
    X, Z = _cg(rng, (M, N)), _cg(rng, (M, N))
    ctx = lib.create(8)
    C = _np(lib.zgemm(ctx, 0, 0, _t(Am), _t(B), alpha=0.7, beta=-0.3, X=_t(X), gamma=1.9, Z=_t(Z),
                      flags=flag | (11 << 8) | (split << 16)))
    ref = 0.7 * (Am @ B) - 0.3 * X + 1.9 * Z
    if flag == 16:
        low = np.tril_indices(M)
        C, ref = C[low], ref[low]
    assert _rel(C, ref) <= 1e-13


@pytest.mark.parametrize("split", [0, 1, 4, 16])
def test_zgemm_lower_gram_with_k_split(lib, split):
    """Gram matrices Y^H Y of a tall block (K = 4000, 200 x 200 output) with
    only the lower triangle formed, as the CholeskyQR and Rayleigh-Ritz steps
    request them: automatic and explicit K splits.  The lower triangle
    matches the product; with a split the strictly upper triangle of C is
    not written (its sentinel survives)."""
    rng = _rng(300 + split)
    K, k = 4000, 200
    Y = _cg(rng, (K, k))
    ctx = lib.create(8)
    sentinel = 7.0 + 7.0j
    C = _t(np.full((k, k), sentinel))
    C = lib.zgemm(ctx, 1, 0, _t(Y), _t(Y), C=C, flags=16 | (split << 16))
    C = _np(C)
    ref = Y.conj().T @ Y
    low = np.tril_indices(k)
    assert np.linalg.norm(C[low] - ref[low]) <= 1e-13 * np.linalg.norm(ref[low])
    if split > 1:
        up = np.triu_indices(k, 1)
        assert np.all(C[up] == sentinel)


def test_zgemm_in_place_epilogue(lib):
    """out aliasing Z (the filter writes Y_{i+1} over Y_{i-1})."""
    import torch
    rng = _rng(10)
    A = _cg(rng, (130, 130))
    Y = _cg(rng, (130, 33))
    P = _cg(rng, (130, 33))
    ctx = lib.create(8)
    Pt = _t(P)
    lib.zgemm(ctx, 0, 0, _t(A), _t(Y), alpha=2.0, beta=-1.0, X=_t(Y), gamma=-0.5, Z=Pt, C=Pt)
    assert _rel(_np(Pt), 2.0 * A @ Y - Y - 0.5 * P) <= 1e-13


# --------------------------------------------------------------------------
# steps of Algorithm 1 against the oracle
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,k,m", [(300, 37, 7), (130, 64, 1), (64, 5, 20)])
def test_filter_matches_oracle(lib, n, k, m):
    p = workloads.make_problem(n, 70 + n)
    rng = _rng(n)
    Y = _cg(rng, (n, k))
    lam = np.sort(p.lam)
    a, b, a0 = float(lam[k]), float(lam[-1] * 1.05), float(lam[0])
    ref = oracle.chebyshev_filter(p.A, Y, m, a, b, a0)
    ctx = lib.create(n)
    Yt = _t(Y)
    lib.filter(ctx, _t(p.A), Yt, m, a, b, a0)
    assert _rel(_np(Yt), ref) <= 1e-12


@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 7, 8, 9, 10, 11, 12])
def test_filter_every_tile_shape_matches_oracle(lib, tile):
    """Every tile configuration of the filter step, those forming complex
    products with three real products (64 x 64 and smaller at two
    workgroups per CU) and those with four, with and without a K split."""
    n, k, m = 300, 37, 5
    p = workloads.make_problem(n, 11)
    Y = _cg(_rng(12), (n, k))
    lam = np.sort(p.lam)
    a, b, a0 = float(lam[k]), float(lam[-1] * 1.05), float(lam[0])
    ref = oracle.chebyshev_filter(p.A, Y, m, a, b, a0)
    for sk in (1, 4):
        ctx = lib.create(n, filter_tile=tile, filter_splitk=sk)
        Yt = _t(Y)
        lib.filter(ctx, _t(p.A), Yt, m, a, b, a0)
        assert _rel(_np(Yt), ref) <= 1e-12, (tile, sk)
        ctx.release()


def test_filter_three_product_form_with_unbalanced_parts(lib):
    """The three-product form cancels in the imaginary part when real parts
    dominate (t1 + t2 = b_r a_i + a_r b_i is formed from two terms of size
    |a_r b_r|).  Its error must still be normwise: relative to the largest
    entry, like the four-product form's.  n = 1100 takes the tall product
    rules (64-wide tiles, K split)."""
    n, k, m = 1100, 70, 3
    rng = _rng(21)
    R = rng.standard_normal((n, n))
    I = rng.standard_normal((n, n))
    A = (R + R.T) / 2 + 1e-6j * (I - I.T) / 2
    A /= np.abs(np.linalg.eigvalsh(A)).max()
    Y = rng.standard_normal((n, k)) + 1e-6j * rng.standard_normal((n, k))
    a, b, a0 = 0.2, 1.05, -1.0
    ref = oracle.chebyshev_filter(A, Y, m, a, b, a0)
    ctx = lib.create(n)
    Yt = _t(Y)
    lib.filter(ctx, _t(A), Yt, m, a, b, a0)
    got = _np(Yt)
    assert _rel(got, ref) <= 1e-12
    assert np.abs((got - ref).imag).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n,k,m", [(300, 37, 7), (1000, 130, 20)])
def test_filter_fp32_against_oracle(lib, n, k, m):
    """Mixed precision: the recurrence in complex FP32 with FP32 accumulation
    agrees with the FP64 oracle to FP32 accuracy (the scaled recurrence keeps
    the iterates O(1), so errors stay near m * eps32)."""
    p = workloads.make_problem(n, 90 + n)
    rng = _rng(n + 1)
    Y = _cg(rng, (n, k))
    lam = np.sort(p.lam)
    a, b, a0 = float(lam[k]), float(lam[-1] * 1.05), float(lam[0])
    ref = oracle.chebyshev_filter(p.A, Y, m, a, b, a0)
    ctx = lib.create(n, precision=1)
    Yt = _t(Y)
    lib.filter(ctx, _t(p.A), Yt, m, a, b, a0)
    err = _rel(_np(Yt), ref)
    assert err <= 2e-5, err
    assert err >= 1e-9  # really computed in FP32


@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 7, 9, 10, 11, 12])
def test_filter_fp32_every_tile_shape(lib, tile):
    """The FP32 filter step in every tile shape (64x48 with 4x1 waves among
    them), with and without a K split, to FP32 accuracy against the FP64
    oracle."""
    n, k, m = 300, 37, 5
    p = workloads.make_problem(n, 13)
    Y = _cg(_rng(14), (n, k))
    lam = np.sort(p.lam)
    a, b, a0 = float(lam[k]), float(lam[-1] * 1.05), float(lam[0])
    ref = oracle.chebyshev_filter(p.A, Y, m, a, b, a0)
    for sk in (1, 4):
        ctx = lib.create(n, precision=1, filter_tile=tile, filter_splitk=sk)
        Yt = _t(Y)
        lib.filter(ctx, _t(p.A), Yt, m, a, b, a0)
        err = _rel(_np(Yt), ref)
        assert 1e-9 <= err <= 2e-5, (tile, sk, err)
        ctx.release()


def test_filter_fp32_tall_rule_takes_48_wide_tile(lib):
    """n = 1100, 44 columns: the tall-product rule picks the 48-wide tile for
    FP32 (64 columns would pad 45 %); the result agrees with the FP64 oracle
    to FP32 accuracy."""
    n, k, m = 1100, 44, 6
    p = workloads.make_problem(n, 15)
    Y = _cg(_rng(16), (n, k))
    lam = np.sort(p.lam)
    a, b, a0 = float(lam[k]), float(lam[-1] * 1.05), float(lam[0])
    ref = oracle.chebyshev_filter(p.A, Y, m, a, b, a0)
    ctx = lib.create(n, precision=1)
    Yt = _t(Y)
    lib.filter(ctx, _t(p.A), Yt, m, a, b, a0)
    err = _rel(_np(Yt), ref)
    assert 1e-9 <= err <= 2e-5, err


@pytest.mark.parametrize("prec", [0, 1])
def test_filter_tall_rule_takes_80_wide_tile(lib, prec):
    """n = 1100, 70 columns: the tall-product rule takes the 80-wide tile
    (one column tile, 12.5 % padding, against 37 % and more for the 64-, 48-
    and 32-wide ones); the result agrees with the oracle (FP64: 1e-12;
    FP32: FP32 accuracy)."""
    n, k, m = 1100, 70, 5
    p = workloads.make_problem(n, 23)
    Y = _cg(_rng(24), (n, k))
    lam = np.sort(p.lam)
    a, b, a0 = float(lam[k]), float(lam[-1] * 1.05), float(lam[0])
    ref = oracle.chebyshev_filter(p.A, Y, m, a, b, a0)
    ctx = lib.create(n, precision=prec)
    Yt = _t(Y)
    lib.filter(ctx, _t(p.A), Yt, m, a, b, a0)
    err = _rel(_np(Yt), ref)
    if prec == 0:
        assert err <= 1e-12, err
    else:
        assert 1e-9 <= err <= 2e-5, err


def test_filter_closed_form_on_diagonal(lib):
    n, k, m = 100, 6, 9
    t = np.linspace(-1.0, 3.0, n)
    a, b, a0 = 0.5, 3.0, -1.0
    rng = _rng(3)
    Y = _cg(rng, (n, k))
    ctx = lib.create(n)
    Yt = _t(Y)
    lib.filter(ctx, _t(np.diag(t).astype(complex)), Yt, m, a, b, a0)
    e, c = (b - a) / 2, (b + a) / 2
    x = (t - c) / e
    cm = np.where(np.abs(x) <= 1, np.cos(m * np.arccos(np.clip(x, -1, 1))),
                  np.sign(x) ** m * np.cosh(m * np.arccosh(np.maximum(np.abs(x), 1))))
    x0 = (a0 - c) / e
    p0 = (-1) ** m * math.cosh(m * math.acosh(-x0))
    assert _rel(_np(Yt), (cm / p0)[:, None] * Y) <= 1e-12


@pytest.mark.parametrize("n,k", [(300, 70), (96, 96), (257, 1), (1000, 40)])
def test_qr_matches_oracle(lib, n, k):
    rng = _rng(n * k)
    Y = _cg(rng, (n, k))
    Qr, R = oracle.householder_qr(Y)
    ctx = lib.create(n)
    Yt = _t(Y)
    lib.qr(ctx, Yt)
    Q = _np(Yt)
    assert np.abs(Q.conj().T @ Q - np.eye(k)).max() <= 1e-13
    # same reflector convention: Q agrees column by column, phases included
    assert _rel(Q, Qr) <= 1e-12


@pytest.mark.parametrize("n,k", [(300, 70), (1000, 130), (64, 64), (257, 1)])
def test_orthonormalize_spans_the_oracle_basis(lib, n, k):
    """The solver's re-orthonormalization (CholeskyQR2) spans the same space
    as the oracle's Householder Q, to working precision."""
    rng = _rng(n + 3 * k)
    Y = _cg(rng, (n, k))
    Qr, _ = oracle.householder_qr(Y)
    ctx = lib.create(n)
    Yt = _t(Y)
    used_hh = lib.orthonormalize(ctx, Yt)
    Q = _np(Yt)
    assert not used_hh
    assert np.abs(Q.conj().T @ Q - np.eye(k)).max() <= 1e-13
    assert np.linalg.norm(Q - Qr @ (Qr.conj().T @ Q), 2) <= 1e-12


def test_orthonormalize_falls_back_on_ill_conditioned_block(lib):
    """cond ~ 1e13: the Gram matrix is not numerically positive definite,
    Householder takes over and the result is still orthonormal and spans the
    dominant directions."""
    rng = _rng(5)
    n, k = 400, 30
    U, _ = np.linalg.qr(_cg(rng, (n, k)))
    V, _ = np.linalg.qr(_cg(rng, (k, k)))
    Y = U @ np.diag(np.logspace(0, -13, k)) @ V
    ctx = lib.create(n)
    Yt = _t(Y)
    used_hh = lib.orthonormalize(ctx, Yt)
    Q = _np(Yt)
    assert used_hh
    assert np.abs(Q.conj().T @ Q - np.eye(k)).max() <= 1e-13
    # the leading directions (singular values >= 1e-4) are captured
    lead = U[:, :9]
    assert np.linalg.norm(lead - Q @ (Q.conj().T @ lead), 2) <= 1e-9


@pytest.mark.parametrize("cond", [1e6, 1e7, 5e7])
@pytest.mark.parametrize("n,k", [(1000, 130), (600, 40)])
def test_orthonormalize_gray_zone(lib, n, k, cond):
    """cond(F) between 1e6 and near the Cholesky breakdown: the Gram
    Cholesky succeeds but two passes alone can leave a visible loss of
    orthogonality.  Whichever path runs (a third CholeskyQR pass or
    Householder), Q is orthonormal to working precision and spans F's
    column space (up to the rounding of F itself, ~eps cond)."""
    rng = _rng(int(math.log10(cond) * 10) + n)
    U, _ = np.linalg.qr(_cg(rng, (n, k)))
    V, _ = np.linalg.qr(_cg(rng, (k, k)))
    Y = U @ np.diag(np.logspace(0, -math.log10(cond), k)) @ V
    ctx = lib.create(n)
    Yt = _t(Y)
    lib.orthonormalize(ctx, Yt)
    Q = _np(Yt)
    assert np.abs(Q.conj().T @ Q - np.eye(k)).max() <= 1e-13
    assert np.linalg.norm(U - Q @ (Q.conj().T @ U), 2) <= 1e-15 * cond * 100


def test_orthonormalize_gray_zone_block_nearly_in_a_subspace(lib):
    """[Y_lock | F] with F's part outside span(Y_lock) graded down to 1e-7
    (the shape of a filtered block next to converged vectors): orthonormal to
    working precision and spanning [Y_lock | U]."""
    rng = _rng(77)
    n, cl, ka = 800, 30, 60
    Yl, _ = np.linalg.qr(_cg(rng, (n, cl)))
    U, _ = np.linalg.qr(_cg(rng, (n, ka)))
    V, _ = np.linalg.qr(_cg(rng, (ka, ka)))
    F = U @ np.diag(np.logspace(0, -7, ka)) @ V + Yl @ _cg(rng, (cl, ka))
    B = np.concatenate([Yl, F], axis=1)
    ctx = lib.create(n)
    Bt = _t(B)
    lib.orthonormalize(ctx, Bt)
    Q = _np(Bt)
    k = cl + ka
    assert np.abs(Q.conj().T @ Q - np.eye(k)).max() <= 1e-13
    # span of [Y_lock | F] is span of [Y_lock | U]
    W = np.concatenate([Yl, U], axis=1)
    assert np.linalg.norm(W - Q @ (Q.conj().T @ W), 2) <= 1e-7


@pytest.mark.parametrize("k", [1, 2, 40, 96, 97, 130, 257, 440])
def test_eigh_matches_oracle(lib, k):
    """Dense random Hermitian matrices: one workgroup up to k = 96, block-ordered
    sweeps above (ragged last block at 97, 130 and 257, an odd block count
    with a phantom block at 97, 130 and 257, 28 blocks at 440)."""
    rng = _rng(k)
    M = _cg(rng, (k, k))
    G = (M + M.conj().T) / 2
    w_ref, Z_ref, _ = oracle.jacobi_eigh(G)
    ctx = lib.create(max(k, 8))
    w, Z = lib.eigh(ctx, _t(G))
    Z = _np(Z)
    gn = np.linalg.norm(G)
    assert np.abs(w - w_ref).max() <= 1e-13 * gn
    assert np.abs(G @ Z - Z * w).max() <= 1e-12 * gn
    assert np.abs(Z.conj().T @ Z - np.eye(k)).max() <= 1e-12
    # eigenvectors of separated eigenvalues agree up to a phase
    gaps = np.minimum(np.diff(np.r_[-np.inf, w_ref]), np.diff(np.r_[w_ref, np.inf]))
    sep = gaps > 1e-3 * gn
    ov = np.abs(np.sum(Z.conj() * Z_ref, axis=0))
    assert np.all(np.abs(ov[sep] - 1) <= 1e-9)


def test_eigh_large_dense_against_library_eigensolver(lib):
    """k = 1000: 63 blocks of 16 (ragged last block, a phantom block), 32
    pairs per round, several block-ordered sweeps before the sparse sweeps
    and the refinement take over.  Eigenvalues against LAPACK's (numpy),
    eigenpairs by their residual and orthogonality."""
    k = 1000
    rng = _rng(1000)
    M = _cg(rng, (k, k))
    G = (M + M.conj().T) / 2
    ref = np.linalg.eigvalsh(G)
    ctx = lib.create(k)
    w, Z = lib.eigh(ctx, _t(G))
    Z = _np(Z)
    gn = np.linalg.norm(G)
    assert np.abs(w - ref).max() <= 1e-13 * gn
    assert np.abs(G @ Z - Z * w).max() <= 1e-12 * gn
    assert np.abs(Z.conj().T @ Z - np.eye(k)).max() <= 1e-12


def test_eigh_clustered_spectrum(lib):
    rng = _rng(44)
    k = 120
    lam = np.sort(np.concatenate([rng.uniform(-1, 1, k - 8), 0.3 + np.linspace(-5e-4, 5e-4, 4),
                                  -0.6 + np.linspace(-5e-4, 5e-4, 4)]))
    Q, _ = np.linalg.qr(_cg(rng, (k, k)))
    G = (Q * lam) @ Q.conj().T
    G = (G + G.conj().T) / 2
    ctx = lib.create(k)
    w, Z = lib.eigh(ctx, _t(G))
    assert np.abs(w - lam).max() <= 1e-14 * k


@pytest.mark.parametrize("k,eps", [(300, 1e-6), (200, 1e-3), (130, 0.0), (64, 1e-6), (96, 1e-4), (24, 1e-8)])
def test_eigh_nearly_diagonal_matches_oracle(lib, k, eps):
    """The projected matrices of late iterations are nearly diagonal: a
    spread diagonal with a tight pair and a Hermitian perturbation of
    relative size eps (the refinement path, for small blocks too), against
    the oracle's Jacobi."""
    rng = _rng(k + 7)
    d = np.sort(rng.uniform(-1, 1, k))
    d[k // 2 + 1] = d[k // 2] + 3e-4  # close pair, still resolved by the coupling ratio
    M = _cg(rng, (k, k))
    G = np.diag(d).astype(complex) + eps * (M + M.conj().T) / 2
    G = (G + G.conj().T) / 2
    w_ref, Z_ref, _ = oracle.jacobi_eigh(G)
    ctx = lib.create(max(k, 8))
    w, Z = lib.eigh(ctx, _t(G))
    Z = _np(Z)
    gn = np.linalg.norm(G)
    assert np.abs(w - w_ref).max() <= 1e-13 * gn
    assert np.abs(G @ Z - Z * w).max() <= 1e-12 * gn
    assert np.abs(Z.conj().T @ Z - np.eye(k)).max() <= 1e-12
    gaps = np.minimum(np.diff(np.r_[-np.inf, w_ref]), np.diff(np.r_[w_ref, np.inf]))
    sep = gaps > 1e-3 * gn
    ov = np.abs(np.sum(Z.conj() * Z_ref, axis=0))
    assert np.all(np.abs(ov[sep] - 1) <= 1e-9)


@pytest.mark.parametrize("n", [200, 64, 333, 777, 1100])
def test_reduce_matches_oracle(lib, n):
    """L, L^{-1} and A = L^{-1} H L^{-H} against the oracle; n above 256
    takes the two-level factorization (outer blocks of 256 columns, the last
    one ragged; the inverse completed by doubling across outer blocks)."""
    p = workloads.make_problem(n, 5 + n)
    L_ref, bad = oracle.cholesky(p.S)
    assert bad == 0
    A_ref = oracle.reduce(p.H, L_ref)
    ctx = lib.create(n)
    lib.reduce(ctx, _t(p.H), _t(p.S))
    A, L, Li = (_np(x) for x in lib.copy_factors(ctx))
    assert np.abs(L - L_ref).max() <= 1e-14
    assert np.all(np.triu(L, 1) == 0) and np.all(np.triu(Li, 1) == 0)
    assert np.abs(Li @ L_ref - np.eye(n)).max() <= 1e-13
    assert _rel(A, A_ref) <= 1e-13
    assert np.array_equal(A, A.conj().T)
    # S == NULL reuses the factor
    lib.reduce(ctx, _t(2 * p.H), None)
    A2 = _np(lib.copy_factors(ctx)[0])
    assert _rel(A2, 2 * A_ref) <= 1e-13


@pytest.mark.parametrize("n,bad", [(150, 100), (600, 400)])
def test_reduce_reports_not_positive_definite(lib, n, bad):
    """The first pivot that is not positive is reported by its column, also
    in a later outer block of the two-level factorization."""
    p = workloads.make_problem(n, 3)
    S = p.S.copy()
    S[bad, bad] = -5.0
    ctx = lib.create(n)
    with pytest.raises(lib.ChfsiError) as e:
        lib.reduce(ctx, _t(p.H), _t(S))
    assert e.value.status == -2
    assert f"column {bad} " in str(e.value)


@pytest.mark.parametrize("n,steps", [(256, 10), (8, 8), (500, 30)])
def test_lanczos_matches_oracle(lib, n, steps):
    p = workloads.make_problem(n, 30 + n)
    v0 = oracle.gauss_block(77, 1, n, 1)[:, 0]
    ref = oracle.lanczos(p.A, steps, v0)
    ctx = lib.create(n)
    got = lib.lanczos(ctx, _t(p.A), steps, 77, 1)
    assert np.allclose(got[:2], ref[:2], rtol=1e-10, atol=1e-12 * abs(ref[1]))
    assert abs(got[2] - ref[2]) <= 1e-8 * abs(ref[2])
    # the bound is safe (exact to rounding when steps == n)
    assert got[2] >= p.lam.max() * (1 - 1e-13)


def test_rayleigh_ritz_and_residuals_match_oracle(lib):
    n, k = 300, 40
    p = workloads.make_problem(n, 17)
    rng = _rng(17)
    Y, _ = np.linalg.qr(_cg(rng, (n, k)))
    mu_ref, Yr = oracle.rayleigh_ritz(p.A, Y)
    ctx = lib.create(n)
    Yt = _t(Y)
    mu, _ = lib.rayleigh_ritz(ctx, _t(p.A), Yt)
    assert np.abs(mu - mu_ref).max() <= 1e-12 * np.abs(p.lam).max()
    Yg = _np(Yt)
    # Ritz vectors agree up to phases (random block: separated Ritz values)
    ov = np.abs(np.sum(Yg.conj() * Yr, axis=0))
    assert np.abs(ov - 1).max() <= 1e-8
    rho_ref = oracle.residuals(p.A, p.L, Yr, mu_ref)
    rho = lib.residuals(ctx, _t(p.A), _t(p.L), _t(Yr), mu_ref)
    assert np.abs(rho - rho_ref).max() <= 1e-12 * rho_ref.max()


# --------------------------------------------------------------------------
# whole solve
# --------------------------------------------------------------------------

def _check_solution(p, evals, X, nev, tol=1e-10):
    hn = _checks.spectral_norm(p.H)
    lam = np.sort(p.lam)
    ok, dmax = _checks.eig_ok(evals, lam[:nev], hn)
    assert ok, dmax
    r = _checks.gen_residuals(p.H, p.S, X, evals)
    assert r.max() <= tol * hn, r.max() / hn
    assert _checks.s_orth_err(p.S, X) <= 1e-12
    Y = _checks.standard_vectors(p.L, X)
    ok, worst, ratio = _checks.subspace_check(Y, _checks.exact_standard_vectors(p.Q, p.lam), p.lam, p.A, evals, nev)
    assert ok, (worst, ratio)


def test_solve_config0_matches_oracle(lib):
    """n=512, nev=51, nex=13, degree 10, tol 1e-10 (the small configuration)."""
    p = workloads.make_problem(512, 0)
    ref = oracle.solve(p.H, p.S, 51, 13, tol=1e-10, degree=10, seed=0)
    ctx = lib.create(512, degree=10, seed=0)
    Hd, Sd = _t(p.H), _t(p.S)
    ev, X, info, st = lib.solve(ctx, Hd, Sd, 51, 13, tol=1e-10)
    assert st == 0 and info["converged"] >= 51
    # the caller's matrices are read, never written
    assert np.array_equal(_np(Hd), p.H) and np.array_equal(_np(Sd), p.S)
    assert np.abs(ev - ref["evals"]).max() <= 1e-12 * 100
    _check_solution(p, ev, _np(X), 51)
    assert info["b_upper"] >= p.lam.max()
    assert info["filter_flops"] > 0 and info["iterations"] > 1


def test_solve_config0_householder_mode_matches_oracle(lib):
    p = workloads.make_problem(512, 0)
    ref = oracle.solve(p.H, p.S, 51, 13, tol=1e-10, degree=10, seed=0)
    ctx = lib.create(512, degree=10, seed=0, qr_mode=1)
    ev, X, info, st = lib.solve(ctx, _t(p.H), _t(p.S), 51, 13, tol=1e-10)
    assert st == 0 and info["qr_householder"] == info["iterations"] + 1
    assert np.abs(ev - ref["evals"]).max() <= 1e-12 * 100
    _check_solution(p, ev, _np(X), 51)


def test_solve_config0_mixed_precision_matches_oracle(lib):
    """FP32 filter + FP64 everything else reaches the same FP64 tolerance."""
    p = workloads.make_problem(512, 0)
    ref = oracle.solve(p.H, p.S, 51, 13, tol=1e-10, degree=10, seed=0)
    ctx = lib.create(512, degree=10, seed=0, precision=1)
    ev, X, info, st = lib.solve(ctx, _t(p.H), _t(p.S), 51, 13, tol=1e-10)
    assert st == 0
    assert info["iterations_fp32"] > 0 and info["filter_launches_fp32"] > 0
    assert np.abs(ev - ref["evals"]).max() <= 1e-12 * 100
    _check_solution(p, ev, _np(X), 51)


@pytest.mark.parametrize("digits", [8, 10])
def test_solve_mixed_precision_switch_below_fp32_floor(lib, digits):
    """A switch below what the FP32 filter can reach (10^-8, 10^-10 h_H):
    the columns stuck at the FP32 rounding floor must turn FP64 together and
    the solve still converge to the FP64 tolerance, in a bounded number of
    iterations (the rule that once moved them one per iteration stalled)."""
    p = workloads.make_problem(512, 0)
    ref = oracle.solve(p.H, p.S, 51, 13, tol=1e-10, degree=10, seed=0)
    ctx64 = lib.create(512, degree=10, seed=0)
    _, _, info64, st64 = lib.solve(ctx64, _t(p.H), _t(p.S), 51, 13, tol=1e-10)
    ctx = lib.create(512, degree=10, seed=0, precision=1, mixed_switch_digits=digits)
    ev, X, info, st = lib.solve(ctx, _t(p.H), _t(p.S), 51, 13, tol=1e-10)
    assert st == 0 and st64 == 0
    assert info["iterations_fp32"] > 0
    assert info["iterations"] <= 2 * info64["iterations"] + 10, (info["iterations"], info64["iterations"])
    assert np.abs(ev - ref["evals"]).max() <= 1e-12 * 100
    _check_solution(p, ev, _np(X), 51)


@pytest.mark.parametrize("case", ["block is the space", "all eigenpairs", "n = 1", "n = 2", "S = I",
                                  "diagonal H, S = I"])
def test_solve_degenerate_cases_against_dense_solver(lib, case):
    """The block spans the whole space (the Lanczos bound is exact for
    n <= its steps, so the damped interval would be empty without its
    guard), the smallest sizes, S = I and an already diagonal H."""
    if case in ("block is the space", "all eigenpairs"):
        p = workloads.make_problem(40, 5)
        H, S = p.H, p.S
        nev, nex = (30, 10) if case == "block is the space" else (40, 0)
    elif case == "n = 1":
        H, S, nev, nex = np.array([[2.5 + 0j]]), np.array([[2.0 + 0j]]), 1, 0
    elif case == "n = 2":
        H, S, nev, nex = np.array([[2.0, 1j], [-1j, 3.0]]), np.eye(2, dtype=complex), 1, 1
    elif case == "S = I":
        p = workloads.make_problem(100, 6)
        H, S, nev, nex = p.A, np.eye(100, dtype=complex), 10, 4
    else:
        H, S, nev, nex = np.diag(np.linspace(-1, 5, 100)).astype(complex), np.eye(100, dtype=complex), 10, 4
    n = H.shape[0]
    ctx = lib.create(n, degree=10, seed=0)
    ev, X, info, st = lib.solve(ctx, _t(H), _t(S), nev, nex, tol=1e-10)
    assert st == 0
    ref = sl.eigh(H, S, eigvals_only=True)[:nev]
    hn = np.linalg.norm(H, 2)
    assert np.abs(ev - ref).max() <= 1e-12 * hn
    Xn = _np(X)
    assert np.linalg.norm(H @ Xn - (S @ Xn) * ev[None, :], axis=0).max() <= 1e-10 * hn


def test_solve_rejects_missing_extra_column(lib):
    p = workloads.make_problem(100, 6)
    ctx = lib.create(100)
    with pytest.raises(lib.ChfsiError) as e:
        lib.solve(ctx, _t(p.H), _t(p.S), 1, 0, tol=1e-10)
    assert e.value.status == -1


def test_solve_ragged_sizes_against_brute_force(lib):
    n, nev, nex = 333, 17, 6
    p = workloads.make_problem(n, 41)
    ctx = lib.create(n, degree=12, seed=3)
    ev, X, info, st = lib.solve(ctx, _t(p.H), _t(p.S), nev, nex, tol=1e-10)
    ref = sl.eigh(p.H, p.S, eigvals_only=True)[:nev]
    hn = _checks.spectral_norm(p.H)
    assert _checks.eig_ok(ev, ref, hn)[0]
    _check_solution(p, ev, _np(X), nev)


def test_solve_warm_sequence(lib):
    """A correlated sequence: S fixed and cached, each solve warm-started from
    the context's state; results checked against a dense library solver."""
    seq = list(workloads.make_sequence(400, 3, 11))
    nev, nex = 30, 6
    ctx = lib.create(400, degree=12, seed=1)
    iters = []
    for ell, p in enumerate(seq):
        S = _t(p.S) if ell == 0 else None
        ev, X, info, st = lib.solve(ctx, _t(p.H), S, nev, nex, tol=1e-10)
        assert st == 0
        assert info["warm_start"] == (1 if ell > 0 else 0)
        hn = _checks.spectral_norm(p.H)
        ref = sl.eigh(p.H, p.S, eigvals_only=True)[:nev]
        assert _checks.eig_ok(ev, ref, hn)[0]
        r = _checks.gen_residuals(p.H, p.S, _np(X), ev)
        assert r.max() <= 1e-10 * hn
        iters.append(info["iterations"])
    cold = lib.create(400, degree=12, seed=1)
    _, _, info_c, _ = lib.solve(cold, _t(seq[-1].H), _t(seq[-1].S), nev, nex, tol=1e-10)
    assert iters[-1] <= info_c["iterations"]


def test_solve_explicit_warm_vectors_with_new_overlap(lib):
    """V_warm given in the generalized space while S is passed again."""
    seq = list(workloads.make_sequence(256, 2, 21))
    nev, nex = 20, 4
    ctx = lib.create(256, degree=10)
    ev0, X0, _, _ = lib.solve(ctx, _t(seq[0].H), _t(seq[0].S), nev, nex)
    ctx2 = lib.create(256, degree=10)
    ev1, X1, info, st = lib.solve(ctx2, _t(seq[1].H), _t(seq[1].S), nev, nex, V_warm=X0)
    assert st == 0 and info["warm_start"] == 1
    p = seq[1]
    hn = _checks.spectral_norm(p.H)
    assert _checks.eig_ok(ev1, sl.eigh(p.H, p.S, eigvals_only=True)[:nev], hn)[0]


def test_solve_error_paths(lib):
    import torch
    p = workloads.make_problem(128, 8)
    ctx = lib.create(128, degree=6, max_iter=2)
    ev, X, info, st = lib.solve(ctx, _t(p.H), _t(p.S), 20, 5, raise_on_noconv=False)
    assert st == -3 and info["converged"] < 20
    c = info["converged"]
    assert np.all(np.isnan(ev[c:]))
    # NaN in H
    H = p.H.copy()
    H[3, 7] = np.nan
    H[7, 3] = np.nan
    ctx2 = lib.create(128, degree=6)
    with pytest.raises(lib.ChfsiError) as e:
        lib.solve(ctx2, _t(H), _t(p.S), 10, 4)
    assert e.value.status == -4
    # the context stays usable after a failure
    ev, X, info, st = lib.solve(ctx2, _t(p.H), _t(p.S), 10, 4)
    assert st == 0
    # invalid arguments
    with pytest.raises(lib.ChfsiError) as e:
        lib.solve(ctx2, _t(p.H), _t(p.S), 100, 40)
    assert e.value.status == -1
    S = p.S.copy()
    S[0, 0] = -1
    with pytest.raises(lib.ChfsiError) as e:
        lib.solve(ctx2, _t(p.H), _t(S), 10, 4)
    assert e.value.status == -2


@pytest.mark.parametrize("precision", [0, 1])
def test_release_returns_device_memory(lib, precision):
    """Release frees a context's device buffers (filter blocks, factors,
    split-K partials, eigensolver scratch; a cold solve with a 110-column
    block takes the block Jacobi sweeps): device free memory after a second
    create / solve / release cycle is not below the memory before it by more
    than 4 MB, far below the tens of MB the context allocates (the first
    cycle loads the code objects; objects of earlier tests are collected
    before each reading, and memory they still free in between only raises
    the second reading)."""
    import gc
    import torch
    p = workloads.make_problem(600, 77)

    def cycle():
        ctx = lib.create(600, degree=12, seed=0, precision=precision)
        ev, X, info, st = lib.solve(ctx, _t(p.H), _t(p.S), 100, 10, tol=1e-10)
        assert st == 0
        del X
        ctx.release()
        torch.cuda.synchronize()

    def free_now():
        gc.collect()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return torch.cuda.mem_get_info()[0]

    cycle()
    free0 = free_now()
    cycle()
    free1 = free_now()
    assert free1 >= free0 - (4 << 20), (free0, free1)


def test_row_major_input_is_not_transposed(lib):
    """A row-major torch tensor must be read as the matrix it represents."""
    import torch
    p = workloads.make_problem(96, 2)
    Hr = torch.from_numpy(p.H.copy(order="C")).cuda()   # row-major
    Sr = torch.from_numpy(p.S.copy(order="C")).cuda()
    ctx = lib.create(96, degree=8)
    ev, X, info, st = lib.solve(ctx, Hr, Sr, 8, 4)
    Xn = _np(X)
    r = _checks.gen_residuals(p.H, p.S, Xn, ev)
    assert r.max() <= 1e-10 * _checks.spectral_norm(p.H)


# --------------------------------------------------------------------------
# full sizes of the benchmark (sampled outputs / properties)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,k,m", [(4000, 440, 20), (4000, 37, 20), (10000, 660, 20)])
def test_filter_full_size_sampled_columns(lib, n, k, m):
    """The filter at benchmark sizes (automatic tile / split choice, as the
    solver launches it); the oracle recomputes a few sampled columns (the
    filter acts on columns independently)."""
    import torch
    rng = _rng(n + k)
    lam = np.sort(workloads.spectrum(n, rng))
    G = torch.from_numpy(_cg(rng, (n, n))).cuda()
    Q, _ = torch.linalg.qr(G)
    del G
    A = (Q * torch.from_numpy(lam).cuda().to(torch.complex128)[None, :]) @ Q.conj().T
    A = (A + A.conj().T) / 2
    del Q
    A = A.mT.contiguous().mT
    Y = _cg(rng, (n, k))
    a, b, a0 = float(lam[min(k, n - 1)]), float(lam[-1] * 1.1), float(lam[0])
    ctx = lib.create(n)
    Yt = _t(Y)
    lib.filter(ctx, A, Yt, m, a, b, a0)
    cols = sorted(set([0, k // 2, k - 1]))
    An = A.cpu().numpy()
    ref = oracle.chebyshev_filter(An, Y[:, cols], m, a, b, a0)
    got = _np(Yt)[:, cols]
    assert _rel(got, ref) <= 1e-12


def test_solve_sequence_configuration_full_size(lib):
    """The benchmark's workload at full size: three problems of the n=4000
    sequence (nev=400, nex=40, degree 20, S fixed and cached, warm starts)
    in the benchmark's launch configuration.  Each solve's eigenvalues
    against a library eigensolver (rocSOLVER through torch) on the step's
    standard-form matrix, which the generator builds directly; residuals of
    the returned pairs; warm solves need fewer iterations than the cold
    one."""
    import torch
    n, nev, nex = 4000, 400, 40
    ctx = lib.create(n, degree=20, seed=0)
    iters = []
    for ell, p in enumerate(workloads.make_sequence_torch(n, 3, 1, device="cuda")):
        ev, X, info, st = lib.solve(ctx, p["H"], p["S"] if ell == 0 else None, nev, nex, tol=1e-10)
        assert st == 0
        assert info["warm_start"] == (1 if ell > 0 else 0)
        ref = torch.linalg.eigvalsh(p["A"]).cpu().numpy()[:nev]
        hn = float(np.abs(torch.linalg.eigvalsh(p["H"]).cpu().numpy()).max())
        ok, dmax = _checks.eig_ok(ev, ref, hn)
        assert ok, (ell, dmax)
        lt = torch.from_numpy(ev).cuda().to(torch.complex128)
        R = p["H"] @ X - (p["S"] @ X) * lt[None, :]
        assert float(torch.linalg.vector_norm(R, dim=0).max()) <= 1e-10 * hn
        iters.append(info["iterations"])
        del X, R
    assert max(iters[1:]) < iters[0]
    ctx.release()


@pytest.fixture(scope="module")
def precision_problem():
    """The precision configuration's problem (n = 10000, spectrum law of the
    small configuration), Gaussian draws on the device."""
    import workloads as w
    p = w.make_problem_torch(10000, 2, device="cuda", rng_kind="device")
    yield p
    del p


def _subspace_full_size(p, X, ev, nev):
    """Subspace angles per cluster-closed group against the constructed
    eigenvectors (Davis-Kahan reading of the 1e-8 rule), on the device."""
    Y = p["L"].conj().T @ X
    ok, worst, ratio = _checks.subspace_check_torch(Y, p["Q"], np.sort(p["lam"]), p["A"], ev, nev)
    assert ok, (worst, ratio)
    return worst


@pytest.mark.parametrize("precision", [0, 1, 2, 3])
def test_solve_precision_configuration_full_size(lib, precision_problem, precision):
    """n=10000, nev=600, nex=60, degree 20, FP64 throughout, mixed precision
    (the filter in complex FP32 until columns approach the tolerance,
    everything else FP64) and the FP32 filter on the Ritz residual (every
    filter product in FP32): every eigenvalue against the spectrum known by
    construction, the generalized residuals of the returned pairs,
    S-orthonormality and subspace angles against the constructed vectors."""
    import torch
    n, nev, nex = 10000, 600, 60
    p = precision_problem
    ctx = lib.create(n, degree=20, seed=0, precision=precision)
    ev, X, info, st = lib.solve(ctx, p["H"], p["S"], nev, nex, tol=1e-10)
    assert st == 0
    assert (info["iterations_fp32"] > 0) == (precision >= 1)
    if precision >= 2:
        assert info["filter_launches_fp32"] == info["filter_launches"]
    lam = np.sort(p["lam"])[:nev]
    H, S = p["H"], p["S"]
    v = torch.ones(n, dtype=torch.complex128, device="cuda")
    for _ in range(50):
        v = H @ v
        v = v / torch.linalg.vector_norm(v)
    hn = float(torch.linalg.vector_norm(H @ v))
    ok, dmax = _checks.eig_ok(ev, lam, hn)
    assert ok, dmax
    lt = torch.from_numpy(ev).cuda().to(torch.complex128)
    R = H @ X - (S @ X) * lt[None, :]
    assert float(torch.linalg.vector_norm(R, dim=0).max()) <= 1e-10 * hn
    G = X.conj().T @ (S @ X)
    assert float((G - torch.eye(nev, dtype=torch.complex128, device="cuda")).abs().max()) <= 1e-12
    del R, G
    _subspace_full_size(p, X, ev, nev)
    ctx.release()


@pytest.mark.parametrize("precision", [0, 1, 2, 3])
def test_solve_full_size_first_problem_of_sequence(lib, precision):
    """n=4000, nev=400, nex=40, degree 20 (the benchmark's sequence, first
    problem: spectrum known by construction)."""
    import torch
    p = workloads.make_problem_torch(4000, 1, device="cuda")
    ctx = lib.create(4000, degree=20, seed=0, precision=precision)
    ev, X, info, st = lib.solve(ctx, p["H"], p["S"], 400, 40, tol=1e-10)
    assert (info["iterations_fp32"] > 0) == (precision >= 1)
    assert st == 0
    lam = np.sort(p["lam"])[:400]
    H, S = p["H"], p["S"]
    v = torch.ones(4000, dtype=torch.complex128, device="cuda")
    for _ in range(50):
        v = H @ v
        v = v / torch.linalg.vector_norm(v)
    hn = float(torch.linalg.vector_norm(H @ v))
    ok, dmax = _checks.eig_ok(ev, lam, hn)
    assert ok, dmax
    lt = torch.from_numpy(ev).cuda().to(torch.complex128)
    R = H @ X - (S @ X) * lt[None, :]
    assert float(torch.linalg.vector_norm(R, dim=0).max()) <= 1e-10 * hn
    G = X.conj().T @ (S @ X)
    assert float((G - torch.eye(400, dtype=torch.complex128, device="cuda")).abs().max()) <= 1e-12
    _subspace_full_size(p, X, ev, 400)
