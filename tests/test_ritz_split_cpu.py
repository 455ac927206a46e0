"""The identity the lower-precision filters rest on, checked on the CPU
against the oracle's filter (eq. (2), FP64): the recurrence is linear in Y,
so for any scalars mu_j its iterates split as Y_i = Y_0 diag(t_i(mu)) + D_i,
t_i the same three-term recurrence on mu_j and D_i the recurrence on
R = A Y_0 - Y_0 diag(mu) with D_0 = 0, D_1 = alpha_0 R and the forcing
alpha_i t_i(mu) R in step i.  The split is exact in exact arithmetic, so in
FP64 the two sides agree to rounding; for Ritz vectors |D| is of the order
of the residual, which is what lets D be formed in lower precision.
"""
import numpy as np
import pytest

import oracle
import workloads


def _schedule(m, a, b, a0):
    # eq. (2) scaled and shifted: (alpha_i, beta_i, gamma_i) of step i
    e, c = (b - a) / 2, (b + a) / 2
    s1 = e / (a0 - c)
    out = [(s1 / e, -s1 / e * c, 0.0)]
    s = s1
    for _ in range(1, m):
        sn = 1.0 / (2.0 / s1 - s)
        out.append((2 * sn / e, -2 * sn / e * c, -s * sn))
        s = sn
    return out


def _split_filter(A, Y0, mu, m, a, b, a0):
    cs = _schedule(m, a, b, a0)
    R = A @ Y0 - Y0 * mu[None, :]
    t_prev, t = np.ones_like(mu), cs[0][0] * mu + cs[0][1]
    D_prev, D = np.zeros_like(R), cs[0][0] * R
    for al, be, ga in cs[1:]:
        D_next = al * (A @ D) + be * D + ga * D_prev + R * (al * t)[None, :]
        t_prev, t = t, al * mu * t + be * t + ga * t_prev
        D_prev, D = D, D_next
    return Y0 * t[None, :] + D, D


@pytest.mark.parametrize("mu_kind", ["ritz", "zero", "random"])
@pytest.mark.parametrize("m", [1, 2, 7])
def test_split_recurrence_reproduces_the_oracle_filter(mu_kind, m):
    n, k = 80, 9
    p = workloads.make_problem(n, 21)
    rng = np.random.default_rng(5)
    Y0 = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    if mu_kind == "ritz":
        Q, _ = np.linalg.qr(Y0)
        mu, Y0 = oracle.rayleigh_ritz(p.A, Q)
    elif mu_kind == "zero":
        mu = np.zeros(k)
    else:
        mu = rng.uniform(-2, 2, k)
    a, b, a0 = 0.3, float(p.lam.max()) * 1.001, float(p.lam.min())
    ref = oracle.chebyshev_filter(p.A, Y0, m, a, b, a0)
    F, _ = _split_filter(p.A, Y0, np.asarray(mu, dtype=float), m, a, b, a0)
    assert np.abs(F - ref).max() <= 1e-12 * np.abs(ref).max()


def test_residual_part_is_small_for_near_eigenvectors():
    """With Ritz vectors of a block near an invariant subspace, |D| / |F| is
    of the order of that block's distance from it (here 1e-6): the part a
    lower precision forms carries only the correction."""
    n, k, m = 120, 10, 8
    p = workloads.make_problem(n, 22)
    order = np.argsort(p.lam)
    rng = np.random.default_rng(6)
    E = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    Y = p.Q[:, order[:k]] + 1e-6 * E / np.linalg.norm(E, axis=0)[None, :]
    Q, _ = np.linalg.qr(Y)
    mu, Yr = oracle.rayleigh_ritz(p.A, Q)
    a, b, a0 = float(mu[-1]), float(p.lam.max()) * 1.001, float(p.lam.min())
    F, D = _split_filter(p.A, Yr, mu, m, a, b, a0)
    ratio = np.abs(D).max() / np.abs(F).max()
    assert 1e-9 < ratio < 1e-4, ratio


def _h(z):
    # complex values with real and imaginary parts rounded to FP16
    return z.real.astype(np.float16).astype(np.float64) + 1j * z.imag.astype(np.float16).astype(np.float64)


@pytest.mark.parametrize("delta", [1e-2, 1e-5])
def test_fp16_operands_on_the_residual_part_keep_errors_relative_to_it(delta):
    """The reading behind the FP16 form, checked in emulation against the
    oracle's FP64 filter: with the products' operands (A and each iterate
    D_i, the latter scaled per column by a power of two) rounded to FP16 and
    everything else exact, the filtered block's error scales with |D| / |F|
    (about delta for Ritz vectors of a block delta away from an invariant
    subspace), while rounding Y_i itself to FP16 errs at FP16's level
    whatever delta is."""
    n, k, m = 150, 12, 8
    p = workloads.make_problem(n, 23)
    order = np.argsort(p.lam)
    rng = np.random.default_rng(7)
    E = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    Q, _ = np.linalg.qr(p.Q[:, order[:k]] + delta * E / np.linalg.norm(E, axis=0)[None, :])
    mu, Y0 = oracle.rayleigh_ritz(p.A, Q)
    a, b, a0 = float(mu[-1]), float(p.lam.max()) * 1.001, float(p.lam.min())
    ref = oracle.chebyshev_filter(p.A, Y0, m, a, b, a0)
    cs = _schedule(m, a, b, a0)
    A16 = _h(p.A)
    # split form, FP16 operands for the residual part
    R = p.A @ Y0 - Y0 * mu[None, :]
    s = 2.0 ** np.ceil(np.log2(np.abs(np.concatenate([R.real, R.imag])).max(axis=0)))
    Rs = R / s[None, :]
    t_prev, t = np.ones_like(mu), cs[0][0] * mu + cs[0][1]
    D_prev, D = np.zeros_like(Rs), cs[0][0] * Rs
    for al, be, ga in cs[1:]:
        D_next = al * (A16 @ _h(D)) + be * D + ga * D_prev + Rs * (al * t)[None, :]
        t_prev, t = t, al * mu * t + be * t + ga * t_prev
        D_prev, D = D, D_next
    F = Y0 * t[None, :] + D * s[None, :]
    # the plain recurrence with FP16 operands
    Yp, Yc = Y0, cs[0][0] * (A16 @ _h(Y0)) + cs[0][1] * Y0
    for al, be, ga in cs[1:]:
        Yp, Yc = Yc, al * (A16 @ _h(Yc)) + be * Yc + ga * Yp
    scale = np.abs(ref).max()
    err_split = np.abs(F - ref).max() / scale
    err_plain = np.abs(Yc - ref).max() / scale
    assert err_plain > 1e-5, err_plain
    assert err_split < 0.1 * delta, (err_split, delta)
