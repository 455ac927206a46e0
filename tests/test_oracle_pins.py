"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: a published known-answer
vector, a factor known by construction, a closed form, brute force on a tiny
input, or an independent library routine.  No expected value here comes from
the GPU library.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg as sl

import oracle
import workloads
from tests import _checks

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


def _cg(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _herm(rng, k):
    M = _cg(rng, (k, k))
    return (M + M.conj().T) / 2


# --------------------------------------------------------------------------
# Counter-based generator (the method's random start block and Lanczos vector)
# --------------------------------------------------------------------------

def test_philox_known_answers():
    """Philox4x32-10 against the Random123 known-answer vectors."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_gauss_block_statistics_and_indexing():
    Y = oracle.gauss_block(7, 3, 400, 250)
    # real and imaginary parts independent N(0, 1): loose 5-sigma bounds
    for part in (Y.real, Y.imag):
        x = part.ravel()
        assert abs(x.mean()) < 5 / math.sqrt(x.size)
        assert abs(x.var() - 1.0) < 5 * math.sqrt(2.0 / x.size)
    assert abs(np.mean(Y.real * Y.imag)) < 5 / math.sqrt(Y.size)
    # column offset selects the same stream entries
    Z = oracle.gauss_block(7, 3, 400, 5, col0=17)
    assert np.array_equal(Z, Y[:, 17:22])
    # streams and seeds differ
    assert not np.allclose(oracle.gauss_block(7, 4, 400, 1), Y[:, :1])
    assert not np.allclose(oracle.gauss_block(8, 3, 400, 1), Y[:, :1])


# --------------------------------------------------------------------------
# Reduction to standard form
# --------------------------------------------------------------------------

def test_cholesky_recovers_constructed_factor():
    p = workloads.make_problem(96, 11)
    L, bad = oracle.cholesky(p.S)
    assert bad == 0
    # the generator's L has a unit diagonal, so it is S's Cholesky factor
    assert np.abs(L - p.L).max() <= 1e-14
    assert np.all(np.triu(L, 1) == 0)


def test_cholesky_against_library_on_general_hpd():
    rng = _rng(3)
    M = _cg(rng, (40, 40))
    S = M @ M.conj().T + 40 * np.eye(40)
    L, bad = oracle.cholesky(S)
    assert bad == 0
    assert np.abs(L - np.linalg.cholesky(S)).max() <= 1e-12


def test_cholesky_reports_first_bad_pivot():
    rng = _rng(4)
    Q, _ = np.linalg.qr(_cg(rng, (6, 6)))
    # leading 3x3 block is PD, so columns 0..2 factor; column 3 fails
    D = np.diag([1.0, 2.0, 3.0, -1.0, 5.0, 6.0]).astype(complex)
    S = D.copy()
    S[:3, :3] = (Q[:3, :3] @ np.diag([1.0, 2.0, 3.0]) @ Q[:3, :3].conj().T) + 3 * np.eye(3)
    L, bad = oracle.cholesky(S)
    assert bad == 4


def test_reduce_recovers_constructed_standard_form():
    p = workloads.make_problem(128, 5)
    L, _ = oracle.cholesky(p.S)
    A = oracle.reduce(p.H, L)
    assert np.abs(A - p.A).max() <= 1e-13 * np.abs(p.A).max()
    assert np.array_equal(A, A.conj().T)


def test_reduce_spectrum_matches_generalized_library_solver():
    rng = _rng(6)
    n = 50
    H = _herm(rng, n)
    M = _cg(rng, (n, n))
    S = M @ M.conj().T / n + np.eye(n)
    L, _ = oracle.cholesky(S)
    A = oracle.reduce(H, L)
    ref = sl.eigh(H, S, eigvals_only=True)
    assert np.abs(np.linalg.eigvalsh(A) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_backtransform_and_lh_times_are_inverse_maps():
    p = workloads.make_problem(64, 9)
    rng = _rng(9)
    Y = _cg(rng, (64, 7))
    X = oracle.backtransform(p.L, Y)
    assert np.abs(p.L.conj().T @ X - Y).max() <= 1e-13
    assert np.abs(oracle.lh_times(p.L, X) - Y).max() <= 1e-13


# --------------------------------------------------------------------------
# Lanczos bound
# --------------------------------------------------------------------------

def test_lanczos_with_n_steps_is_exact():
    rng = _rng(12)
    n = 8
    A = _herm(rng, n)
    ev = np.linalg.eigvalsh(A)
    tmin, tmax, b = oracle.lanczos(A, n, _cg(rng, (n,)))
    assert abs(tmin - ev[0]) <= 1e-12 and abs(tmax - ev[-1]) <= 1e-12
    assert abs(b - ev[-1]) <= 1e-10


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_lanczos_upper_bound_is_safe(seed):
    p = workloads.make_problem(256, 100 + seed)
    tmin, tmax, b = oracle.lanczos(p.A, 10, oracle.gauss_block(seed, 1, 256, 1)[:, 0])
    lam_max = p.lam.max()
    assert b >= lam_max
    assert tmax <= lam_max + 1e-12 and tmin >= p.lam.min() - 1e-12


# --------------------------------------------------------------------------
# Chebyshev filter (closed form of the scaled Chebyshev polynomial)
# --------------------------------------------------------------------------

def cheb(m, x):
    """C_m(x) from its trigonometric / hyperbolic closed form."""
    x = np.asarray(x, dtype=float)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1
    out[inside] = np.cos(m * np.arccos(x[inside]))
    big = x > 1
    out[big] = np.cosh(m * np.arccosh(x[big]))
    small = x < -1
    out[small] = (-1) ** m * np.cosh(m * np.arccosh(-x[small]))
    return out


def p_closed(m, t, a, b, a0):
    e = (b - a) / 2
    c = (b + a) / 2
    return cheb(m, (np.asarray(t) - c) / e) / cheb(m, np.array([(a0 - c) / e]))[0]


@pytest.mark.parametrize("m", [1, 2, 3, 7, 20])
def test_filter_matches_closed_form_on_diagonal(m):
    rng = _rng(20 + m)
    n, k = 60, 5
    a, b, a0 = -0.2, 3.0, -1.5
    t = np.sort(rng.uniform(-1.5, 3.0, n))
    t[0] = a0  # p(a0) must be exactly 1
    Y = _cg(rng, (n, k))
    F = oracle.chebyshev_filter(np.diag(t).astype(complex), Y, m, a, b, a0)
    p = p_closed(m, t, a, b, a0)
    assert abs(p[0] - 1.0) <= 1e-14
    err = np.abs(F - p[:, None] * Y).max() / np.abs(p[:, None] * Y).max()
    assert err <= 1e-13
    # on [a, b] the filter is bounded by 1/|C_m(t0)|
    inside = (t >= a) & (t <= b)
    bound = 1.0 / abs(cheb(m, np.array([(a0 - (a + b) / 2) / ((b - a) / 2)]))[0])
    assert np.all(np.abs(F[inside]) <= bound * np.abs(Y[inside]) * (1 + 1e-12))


def test_filter_commutes_with_unitary_similarity():
    rng = _rng(31)
    n, k, m = 48, 6, 9
    Q, _ = np.linalg.qr(_cg(rng, (n, n)))
    lam = np.sort(rng.uniform(-1, 10, n))
    A = (Q * lam) @ Q.conj().T
    A = (A + A.conj().T) / 2
    Y = _cg(rng, (n, k))
    a, b, a0 = 2.0, 10.5, -1.0
    F = oracle.chebyshev_filter(A, Y, m, a, b, a0)
    ref = Q @ (p_closed(m, lam, a, b, a0)[:, None] * (Q.conj().T @ Y))
    assert np.abs(F - ref).max() / np.abs(ref).max() <= 1e-12


# --------------------------------------------------------------------------
# Householder QR
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,k", [(40, 40), (100, 13), (7, 1)])
def test_householder_qr_properties(n, k):
    rng = _rng(n + k)
    Y = _cg(rng, (n, k))
    Q, R = oracle.householder_qr(Y)
    assert np.abs(Q.conj().T @ Q - np.eye(k)).max() <= 1e-14 * k
    assert np.abs(Q @ R - Y).max() <= 1e-14 * k * np.abs(Y).max()
    assert np.all(np.tril(R, -1) == 0)
    assert np.all(np.diag(R).imag == 0)
    # R is unique up to the phases of its rows: compare moduli with LAPACK's
    R2 = np.linalg.qr(Y, mode="r")
    assert np.abs(np.abs(R) - np.abs(R2)).max() <= 1e-12 * np.abs(R2).max()


def test_householder_qr_graded_columns():
    """Filtered blocks are graded (column norms spread over many decades);
    the span must still be exact to working precision."""
    rng = _rng(77)
    n, k = 80, 10
    U, _ = np.linalg.qr(_cg(rng, (n, k)))
    # column norms from 1 down to 1e-18: Householder QR is column-wise
    # backward stable, so each column direction survives to working precision
    Y = U @ np.diag(10.0 ** (-2.0 * np.arange(k)))
    Q, R = oracle.householder_qr(Y)
    assert np.abs(Q.conj().T @ Q - np.eye(k)).max() <= 1e-13
    # span(Q) == span(U), and column j of Q is column j of U up to a phase
    assert np.linalg.norm(Q - U @ (U.conj().T @ Q), 2) <= 1e-13
    assert np.abs(np.abs(np.sum(Q.conj() * U, axis=0)) - 1).max() <= 1e-13


# --------------------------------------------------------------------------
# Jacobi eigensolver and Rayleigh-Ritz
# --------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2, 5, 40])
def test_jacobi_against_library(k):
    rng = _rng(50 + k)
    G = _herm(rng, k)
    w, Z, sweeps = oracle.jacobi_eigh(G)
    ref = np.linalg.eigvalsh(G)
    assert np.abs(w - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    assert np.abs(G @ Z - Z * w).max() <= 1e-13 * np.abs(G).max()
    assert np.abs(Z.conj().T @ Z - np.eye(k)).max() <= 1e-13
    assert np.all(np.diff(w) >= 0)


def test_jacobi_two_by_two_closed_form():
    g = 0.3 - 0.4j
    G = np.array([[1.0, g], [np.conj(g), -2.0]])
    w, Z, _ = oracle.jacobi_eigh(G)
    mid, rad = -0.5, math.sqrt(1.5 ** 2 + abs(g) ** 2)
    assert abs(w[0] - (mid - rad)) <= 1e-15 and abs(w[1] - (mid + rad)) <= 1e-15


def test_jacobi_known_spectrum_with_cluster():
    rng = _rng(5)
    k = 30
    lam = np.sort(np.concatenate([rng.uniform(-1, 1, k - 4), 0.25 + np.linspace(-5e-4, 5e-4, 4)]))
    Q, _ = np.linalg.qr(_cg(rng, (k, k)))
    G = (Q * lam) @ Q.conj().T
    G = (G + G.conj().T) / 2
    w, Z, _ = oracle.jacobi_eigh(G)
    assert np.abs(w - lam).max() <= 1e-14 * k


def test_jacobi_diagonal_and_repeated():
    w, Z, sweeps = oracle.jacobi_eigh(np.diag([3.0, -1.0, 3.0, 2.0]).astype(complex))
    assert list(w) == [-1.0, 2.0, 3.0, 3.0]
    assert sweeps == 0
    # ties keep index order: eigenvalue 3 of column 0 before column 2
    assert abs(Z[0, 2]) == 1.0 and abs(Z[2, 3]) == 1.0
    w, Z, _ = oracle.jacobi_eigh(np.eye(5, dtype=complex))
    assert np.all(w == 1.0)


def test_rayleigh_ritz_on_invariant_subspace():
    p = workloads.make_problem(120, 21)
    rng = _rng(21)
    k = 9
    idx = np.argsort(p.lam)[:k]
    U, _ = np.linalg.qr(_cg(rng, (k, k)))
    Y = p.Q[:, idx] @ U
    mu, Yr = oracle.rayleigh_ritz(p.A, Y)
    assert np.abs(mu - np.sort(p.lam)[:k]).max() <= 1e-13 * 100
    assert np.abs(p.A @ Yr - Yr * mu).max() <= 1e-12


def test_residuals_equal_generalized_residuals():
    p = workloads.make_problem(70, 22)
    rng = _rng(22)
    Y, _ = np.linalg.qr(_cg(rng, (70, 4)))
    mu = rng.uniform(-1, 1, 4)
    rho = oracle.residuals(p.A, p.L, Y, mu)
    X = sl.solve_triangular(p.L.conj().T, Y, lower=False)
    ref = _checks.gen_residuals(p.H, p.S, X, mu)
    assert np.abs(rho - ref).max() <= 1e-12 * ref.max()


# --------------------------------------------------------------------------
# Whole solve (Algorithm 1)
# --------------------------------------------------------------------------

def _check_solution(p, res, nev, tol=1e-10):
    hn = _checks.spectral_norm(p.H)
    lam = np.sort(p.lam)
    ok, dmax = _checks.eig_ok(res["evals"], lam[:nev], hn)
    assert ok, dmax
    X = res["X"]
    r = _checks.gen_residuals(p.H, p.S, X, res["evals"])
    assert r.max() <= tol * hn, r.max() / hn
    assert _checks.s_orth_err(p.S, X) <= 1e-12
    Y = _checks.standard_vectors(p.L, X)
    ok, worst, ratio = _checks.subspace_check(Y, _checks.exact_standard_vectors(p.Q, p.lam), p.lam, p.A,
                                              res["evals"], nev)
    assert ok, (worst, ratio)


def test_solve_tiny_against_brute_force():
    n, nev, nex = 48, 6, 4
    p = workloads.make_problem(n, 40)
    res = oracle.solve(p.H, p.S, nev, nex, degree=8, seed=1)
    assert res["info"]["status"] == 0
    ref = sl.eigh(p.H, p.S, eigvals_only=True)[:nev]
    assert np.abs(res["evals"] - ref).max() <= 1e-12 * np.abs(ref).max() + 1e-13
    _check_solution(p, res, nev)


def test_solve_config0_shape():
    """n=512, nev=51, nex=13, degree 10, tol 1e-10, spectrum known."""
    p = workloads.make_problem(512, 0)
    res = oracle.solve(p.H, p.S, 51, 13, tol=1e-10, degree=10, seed=0)
    info = res["info"]
    assert info["status"] == 0 and info["converged"] >= 51
    assert info["b_upper"] >= p.lam.max()
    assert info["h_H"] <= _checks.spectral_norm(p.H) * (1 + 1e-12)
    assert np.all(np.diff(res["evals"]) >= 0)
    _check_solution(p, res, 51)


def test_solve_warm_start_sequence():
    seq = list(workloads.make_sequence(160, 3, 3))
    nev, nex = 16, 4
    prev = None
    for ell, p in enumerate(seq):
        cold = oracle.solve(p.H, p.S, nev, nex, degree=10, seed=5)
        assert cold["info"]["status"] == 0
        ref = sl.eigh(p.H, p.S, eigvals_only=True)[:nev]
        hn = _checks.spectral_norm(p.H)
        assert _checks.eig_ok(cold["evals"], ref, hn)[0]
        if prev is not None:
            Xw = sl.solve_triangular(p.L.conj().T, prev["Y"], lower=False)
            warm = oracle.solve(p.H, p.S, nev, nex, degree=10, seed=5, V_warm=Xw,
                                bounds=[prev["info"]["a0"], prev["info"]["a"]])
            assert warm["info"]["status"] == 0
            assert _checks.eig_ok(warm["evals"], ref, hn)[0]
            r = _checks.gen_residuals(p.H, p.S, warm["X"], warm["evals"])
            assert r.max() <= 1e-10 * hn
            assert warm["info"]["iterations"] <= cold["info"]["iterations"]
            prev = warm
        else:
            prev = cold


def test_solve_reports_not_positive_definite():
    p = workloads.make_problem(32, 1)
    S = p.S.copy()
    S[5, 5] = -1.0
    res = oracle.solve(p.H, S, 4, 2)
    assert res["info"]["status"] == -2 and res["info"]["bad_column"] <= 5


def test_solve_reports_no_convergence_with_prefix():
    p = workloads.make_problem(128, 2)
    res = oracle.solve(p.H, p.S, 12, 4, degree=4, max_iter=2)
    info = res["info"]
    assert info["status"] == -3 and info["converged"] < 12
    c = info["converged"]
    assert np.all(np.isfinite(res["evals"][:c])) and np.all(np.isnan(res["evals"][c:]))


def test_solve_rejects_bad_arguments():
    p = workloads.make_problem(16, 1)
    assert oracle.solve(p.H, p.S, 10, 10)["info"]["status"] == -1
    assert oracle.solve(p.H, p.S, 0, 2)["info"]["status"] == -1
    assert oracle.solve(p.H, p.S, 2, 2, tol=0.0)["info"]["status"] == -1
    # no extra column while the block is not the whole space
    assert oracle.solve(p.H, p.S, 2, 0)["info"]["status"] == -1


@pytest.mark.parametrize("case", ["n = 1", "n = 2", "block is the space"])
def test_solve_degenerate_sizes_against_dense_solver(case):
    """The Lanczos bound is exact for n at most its steps, so with the block
    spanning the space the damped interval would be empty; the solve must
    still give the dense solver's eigenpairs."""
    if case == "n = 1":
        H, S, nev, nex = np.array([[2.5 + 0j]]), np.array([[2.0 + 0j]]), 1, 0
    elif case == "n = 2":
        H, S, nev, nex = np.array([[2.0, 1j], [-1j, 3.0]]), np.eye(2, dtype=complex), 1, 1
    else:
        p = workloads.make_problem(40, 5)
        H, S, nev, nex = p.H, p.S, 30, 10
    res = oracle.solve(H, S, nev, nex, tol=1e-10, degree=10, seed=0)
    assert res["info"]["status"] == 0
    ref = sl.eigh(H, S, eigvals_only=True)[:nev]
    hn = np.linalg.norm(H, 2)
    assert np.abs(res["evals"] - ref).max() <= 1e-12 * hn
    X = res["X"]
    assert np.linalg.norm(H @ X - (S @ X) * res["evals"][None, :], axis=0).max() <= 1e-10 * hn
