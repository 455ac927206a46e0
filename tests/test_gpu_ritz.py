"""The filter on the Ritz residual against the oracle (precision 2: its
products in complex FP32; precision 3: with FP16 operands).

The recurrence of eq. (2) is linear in Y, so for Ritz vectors Y_0 of A with
Ritz values mu its iterates split as Y_i = Y_0 diag(t_i(mu)) + D_i: t_i the
same recurrence on the scalars mu_j, D_i the recurrence on the residual
A Y_0 - Y_0 diag(mu) (D_0 = 0).  The library forms D in complex FP32 and
the rest in FP64.  Exact arithmetic gives the oracle's p(A) Y_0 for any mu;
in floating point the FP32 rounding is relative to |D|, not to |Y_i|.

Tolerances (element by element, each column scaled by its largest entry in
the oracle's result): the plain FP32 filter at these sizes is off by a few
1e-6 (2^-24 per operation over n-term sums and m steps); the split form's
error is that level times |D|/|F|, which is about the perturbation delta of
near-converged vectors: ~5e-12 at delta = 1e-6, bound 1e-10; with FP16
operands (precision 3; 2^-11 per rounding) the level is ~5e-3, ~6e-9 at
delta = 1e-6 (an emulation of the same arithmetic on the CPU), bound 1e-7;
for vectors that are not a Ritz basis (|D| ~ |F|) the bounds are the plain
levels, 5e-5 (FP32) and 5e-2 (FP16).
"""
import numpy as np
import pytest

import oracle
import workloads
from tests import _checks

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    a = np.asarray(a, dtype=np.complex128)
    return torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda").mT


def _np(t):
    return t.detach().cpu().numpy()


def _colerr(F, ref):
    return float((np.abs(F - ref).max(axis=0) / np.abs(ref).max(axis=0)).max())


def _ritz_block(n, k, delta, seed):
    """Ritz vectors (oracle Rayleigh-Ritz) of the constructed eigenvectors of
    the k lowest eigenvalues, perturbed by delta (relative per column)."""
    p = workloads.make_problem(n, seed)
    order = np.argsort(p.lam)
    rng = np.random.default_rng(seed + 100)
    E = (rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))) / np.sqrt(2 * n)
    Y = p.Q[:, order[:k]] + delta * E
    Q, _ = np.linalg.qr(Y)
    mu, Yr = oracle.rayleigh_ritz(p.A, Q)
    return p, mu, Yr, p.A @ Yr


# (precision, n, k, tile, split): one tile of each family the FP32 step
# takes, with and without a K split (the forcing term is added in the step's
# epilogue or in the split-K combination), ragged row and column tails; the
# FP16 step's three tile shapes (0: automatic, 128 x 64; 1: 64 x 64; 6:
# 128 x 128) with and without splits
CASES = [(2, 700, 70, 0, 0), (2, 700, 70, 1, 1), (2, 700, 70, 1, 4), (2, 650, 45, 10, 1), (2, 650, 45, 10, 3),
         (2, 900, 150, 12, 2), (2, 900, 150, 11, 1), (2, 900, 150, 3, 2),
         (3, 700, 70, 0, 0), (3, 700, 70, 0, 1), (3, 700, 70, 0, 4), (3, 650, 45, 0, 3), (3, 900, 150, 0, 2),
         (3, 1100, 130, 0, 0), (3, 700, 70, 1, 0), (3, 650, 45, 1, 3), (3, 900, 150, 6, 2), (3, 1100, 130, 6, 0)]
BOUND = {2: 1e-10, 3: 1e-7}
# outer iterations allowed beyond the FP64 solve's (CPU emulations of both
# forms took the FP64 count at n = 600 and 1500)
SLACK = {2: 1, 3: 3}


@pytest.mark.parametrize("prec,n,k,tile,sk", CASES)
def test_filter_ritz_keeps_fp64_accuracy_on_ritz_vectors(lib, prec, n, k, tile, sk):
    m = 10
    p, mu, Yr, AY = _ritz_block(n, k, 1e-6, 3)
    a, b, a0 = float(mu[-1]), float(p.lam.max()) * 1.0001, float(p.lam.min())
    ref = oracle.chebyshev_filter(p.A, Yr, m, a, b, a0)
    ctx = lib.create(n, precision=prec, filter_tile=tile, filter_splitk=sk)
    print(f"filter_ritz precision={prec} n={n} k={k} tile={tile} split={sk}", flush=True)
    Y = _t(Yr)
    lib.filter_ritz(ctx, _t(p.A), Y, _t(AY), mu, m, a, b, a0)
    err = _colerr(_np(Y), ref)
    ctx32 = lib.create(n, precision=1, filter_tile=tile, filter_splitk=sk)
    Y32 = _t(Yr)
    lib.filter(ctx32, _t(p.A), Y32, m, a, b, a0)
    err32 = _colerr(_np(Y32), ref)
    assert err <= BOUND[prec], (err, err32)
    assert err32 >= 1e-8, err32  # the plain FP32 filter cannot reach it
    ctx.release()
    ctx32.release()


@pytest.mark.parametrize("prec", [2, 3])
@pytest.mark.parametrize("mu_kind", ["zero", "shifted"])
def test_filter_ritz_is_exact_for_any_mu(lib, mu_kind, prec):
    """Y_0 not a Ritz basis and mu not its Ritz values: the split is still
    the filter (errors at the plain FP32 level)."""
    n, k, m = 600, 40, 8
    p = workloads.make_problem(n, 4)
    rng = np.random.default_rng(9)
    Y0 = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    mu = np.zeros(k) if mu_kind == "zero" else np.linspace(-0.5, 0.5, k)
    a, b, a0 = 0.2, float(p.lam.max()) * 1.0001, float(p.lam.min())
    ref = oracle.chebyshev_filter(p.A, Y0, m, a, b, a0)
    ctx = lib.create(n, precision=prec)
    Y = _t(Y0)
    lib.filter_ritz(ctx, _t(p.A), Y, _t(p.A @ Y0), mu, m, a, b, a0)
    assert _colerr(_np(Y), ref) <= {2: 5e-5, 3: 5e-2}[prec]
    ctx.release()


@pytest.mark.parametrize("prec", [2, 3])
def test_filter_ritz_degree_one(lib, prec):
    """m = 1: no lower-precision product at all, Y_1 = Y_0 t_1(mu) + alpha_0 R."""
    n, k = 300, 20
    p, mu, Yr, AY = _ritz_block(n, k, 1e-3, 5)
    a, b, a0 = float(mu[-1]), float(p.lam.max()) * 1.0001, float(p.lam.min())
    ref = oracle.chebyshev_filter(p.A, Yr, 1, a, b, a0)
    ctx = lib.create(n, precision=prec)
    Y = _t(Yr)
    lib.filter_ritz(ctx, _t(p.A), Y, _t(AY), mu, 1, a, b, a0)
    assert _colerr(_np(Y), ref) <= 1e-10
    ctx.release()


def test_filter_ritz_rejects_bad_arguments(lib):
    import torch
    n = 64
    ctx = lib.create(n)
    A = torch.eye(n, dtype=torch.complex128, device="cuda")
    Y = torch.zeros((n, 4), dtype=torch.complex128, device="cuda")
    with pytest.raises(ValueError):
        lib.filter_ritz(ctx, A, Y, Y.clone(), np.zeros(3), 4, 0.0, 1.0, -1.0)
    with pytest.raises(lib.ChfsiError):
        lib.filter_ritz(ctx, A, Y, Y.clone(), np.zeros(4), 4, 1.0, 1.0, -1.0)  # b = a
    with pytest.raises(lib.ChfsiError):
        lib.filter_ritz(ctx, A, Y, Y.clone(), np.zeros(4), 0, 0.0, 1.0, -1.0)  # m = 0
    ctx.release()


@pytest.mark.parametrize("prec", [2, 3])
def test_solve_config0_ritz_filter_matches_oracle(lib, prec):
    """n=512, nev=51, nex=13, degree 10: every filter product in FP32 (or
    with FP16 operands), the same FP64 tolerance and no more outer
    iterations than the FP64 solve."""
    p = workloads.make_problem(512, 0)
    ref = oracle.solve(p.H, p.S, 51, 13, tol=1e-10, degree=10, seed=0)
    ctx64 = lib.create(512, degree=10, seed=0)
    _, _, info64, st64 = lib.solve(ctx64, _t(p.H), _t(p.S), 51, 13, tol=1e-10)
    ctx = lib.create(512, degree=10, seed=0, precision=prec)
    ev, X, info, st = lib.solve(ctx, _t(p.H), _t(p.S), 51, 13, tol=1e-10)
    assert st == 0 and st64 == 0
    assert info["iterations_fp32"] == info["iterations"]
    assert info["filter_launches_fp32"] == info["filter_launches"]
    assert info["iterations"] <= info64["iterations"] + SLACK[prec], (info["iterations"], info64["iterations"])
    assert np.abs(ev - ref["evals"]).max() <= 1e-12 * 100
    X = _np(X)
    hn = _checks.spectral_norm(p.H)
    assert _checks.gen_residuals(p.H, p.S, X, ev).max() <= 1e-10 * hn
    assert _checks.s_orth_err(p.S, X) <= 1e-12
    Y = _checks.standard_vectors(p.L, X)
    ok, worst, ratio = _checks.subspace_check(Y, _checks.exact_standard_vectors(p.Q, p.lam), p.lam, p.A, ev, 51)
    assert ok, (worst, ratio)


@pytest.mark.parametrize("prec", [2, 3])
def test_solve_ritz_filter_warm_sequence(lib, prec):
    """A correlated sequence, S fixed and cached, each solve warm-started
    from the context's kept block (whose first iteration, not a Ritz basis
    of the new matrix, runs the plain FP32 filter): eigenvalues against a
    dense library solver, residuals, and no more iterations than FP64."""
    import scipy.linalg as sl
    seq = list(workloads.make_sequence(400, 3, 11))
    nev, nex = 30, 6
    ctx = lib.create(400, degree=12, seed=1, precision=prec)
    ctx64 = lib.create(400, degree=12, seed=1)
    for ell, p in enumerate(seq):
        S = _t(p.S) if ell == 0 else None
        ev, X, info, st = lib.solve(ctx, _t(p.H), S, nev, nex, tol=1e-10)
        _, _, info64, st64 = lib.solve(ctx64, _t(p.H), S, nev, nex, tol=1e-10)
        assert st == 0 and st64 == 0
        assert info["warm_start"] == (1 if ell > 0 else 0)
        assert info["iterations_fp32"] == info["iterations"]
        assert info["iterations"] <= info64["iterations"] + SLACK[prec], (ell, info["iterations"], info64["iterations"])
        hn = _checks.spectral_norm(p.H)
        ref = sl.eigh(p.H, p.S, eigvals_only=True)[:nev]
        assert _checks.eig_ok(ev, ref, hn)[0]
        assert _checks.gen_residuals(p.H, p.S, _np(X), ev).max() <= 1e-10 * hn


def test_batch_rejects_fp16_operands(lib):
    with pytest.raises(lib.ChfsiError):
        lib.Batch([64, 80], use_graph=False, degree=4, seed=0, precision=3)
