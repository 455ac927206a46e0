"""Acceptance checks shared by the oracle pins and the GPU parity tests.

* eigenvalues: |dlam| <= 1e-10 |lam|  or  |dlam| <= 1e-12 ||H||_2 (a purely
  relative bound is out of reach for eigenvalues near zero: the backward
  stable floor is ~ sqrt(n) eps ||A|| in absolute terms);
* residuals:   ||H x - lam S x||_2 <= 1e-10 ||H||_2 (the paper's 1e-10);
* vectors: S-orthonormality, and subspace angles compared per group of
  eigenvalues closed under clusters (groups split only where the gap exceeds
  2e-3): sin angle <= max(1e-8, ||R_G||_F / delta_G), the Davis-Kahan bound
  for the group's residual R_G and its gap delta_G to the rest of the
  spectrum.  A group that straddles the nev-th eigenvalue is compared with
  the full cluster's exact span.
"""
import numpy as np
import scipy.linalg as sl

CLUSTER_GAP = 2e-3


def eig_ok(got, ref, hnorm, rel=1e-10, abs_floor=1e-12):
    d = np.abs(np.asarray(got) - np.asarray(ref))
    ok = (d <= rel * np.abs(ref)) | (d <= abs_floor * hnorm)
    return bool(np.all(ok)), float(d.max())


def gen_residuals(H, S, X, lam):
    R = H @ X - (S @ X) * np.asarray(lam)[None, :]
    return np.linalg.norm(R, axis=0)


def s_orth_err(S, X):
    k = X.shape[1]
    return float(np.abs(X.conj().T @ S @ X - np.eye(k)).max())


def groups(lam_all, nev, gap=CLUSTER_GAP):
    """Index groups over [0, nev) split where consecutive eigenvalues differ
    by more than ``gap``; the last group is extended past nev (its ``full``
    range) while the spectrum continues within ``gap``."""
    lam_all = np.sort(lam_all)
    out = []
    start = 0
    for i in range(1, nev + 1):
        if i == nev or lam_all[i] - lam_all[i - 1] > gap:
            end = i
            full_end = end
            while full_end < len(lam_all) and lam_all[full_end] - lam_all[full_end - 1] <= gap:
                full_end += 1
            out.append((start, end, full_end))
            start = i
    return out


def subspace_check(Y, Y_exact_all, lam_all, A, mu, nev):
    """Y: standard-form computed vectors (n x nev, orthonormal); Y_exact_all:
    exact standard-form eigenvectors sorted ascending (n x >= nev+extra);
    A: standard-form matrix.  Returns (ok, worst raw sin angle, worst ratio
    of the angle to its allowed bound)."""
    lam_all = np.sort(lam_all)
    worst = 0.0
    ratio = 0.0
    ok = True
    for (s, e, fe) in groups(lam_all, nev):
        YG = Y[:, s:e]
        E = Y_exact_all[:, s:fe]
        P = YG - E @ (E.conj().T @ YG)
        sin = float(np.linalg.norm(P, 2))
        RG = A @ YG - YG * np.asarray(mu[s:e])[None, :]
        lo = lam_all[s - 1] if s > 0 else -np.inf
        hi = lam_all[fe] if fe < len(lam_all) else np.inf
        delta = min(np.min(mu[s:e]) - lo, hi - np.max(mu[s:e]))
        bound = max(1e-8, float(np.linalg.norm(RG)) / max(delta, 1e-300))
        worst = max(worst, sin)
        ratio = max(ratio, sin / bound)
        if sin > bound:
            ok = False
    return ok, worst, ratio


def standard_vectors(L, X):
    """Y = L^H X."""
    return L.conj().T @ X


def exact_standard_vectors(Q, lam):
    idx = np.argsort(lam, kind="stable")
    return Q[:, idx]


def spectral_norm(M):
    return float(sl.norm(M, 2))


def subspace_check_torch(Y, Q_sorted, lam_sorted, A, mu, nev):
    """subspace_check on the device (torch tensors Y n x nev, Q_sorted n x N
    the exact standard-form eigenvectors in ascending order, A n x n; host
    arrays lam_sorted, mu), for the full-size tests."""
    import torch
    lam_sorted = np.asarray(lam_sorted)
    mu = np.asarray(mu)
    worst = 0.0
    ratio = 0.0
    ok = True
    for (s, e, fe) in groups(lam_sorted, nev):
        YG = Y[:, s:e]
        E = Q_sorted[:, s:fe]
        P = YG - E @ (E.conj().T @ YG)
        sin = float(torch.linalg.matrix_norm(P, ord=2))
        m = torch.from_numpy(mu[s:e]).to(device=Y.device, dtype=Y.dtype)
        RG = A @ YG - YG * m[None, :]
        lo = lam_sorted[s - 1] if s > 0 else -np.inf
        hi = lam_sorted[fe] if fe < len(lam_sorted) else np.inf
        delta = min(np.min(mu[s:e]) - lo, hi - np.max(mu[s:e]))
        bound = max(1e-8, float(torch.linalg.matrix_norm(RG)) / max(delta, 1e-300))
        worst = max(worst, sin)
        ratio = max(ratio, sin / bound)
        if sin > bound:
            ok = False
    return ok, worst, ratio
