"""Seeded synthetic inputs shaped like the paper's FLAPW eigenproblems.

This module only builds inputs (matrices with a spectrum known by
construction, sequences of correlated problems); it holds none of the
solver's arithmetic.  Both the CPU oracle's tests and the GPU library's
tests and benchmark draw their inputs from here, so that the two sides see
the same arrays.

The FLEUR matrices the paper solves (Au98Ag10, Na15Cl14Li; Table 1) are not
available, so every workload is synthetic:

* spectrum law: the lowest 20 % of the eigenvalues uniform in [-1, 0.5]
  holding 5 tight clusters of 4 members spread evenly over a width of 1e-3,
  the rest log-uniform in [0.5, 100];
* A = Q diag(lam) Q^H with Q the unitary factor of a complex Gaussian matrix;
* S = L L^H with L = I + 0.05 tril(G, -1)/sqrt(n), G complex Gaussian of unit
  variance; H = L A L^H (all symmetrized so they are exactly Hermitian);
* sequences: A_{l+1} = A_l + 1e-4 ||A_l||_2 (E + E^H)/2 with E a complex
  Gaussian matrix scaled to unit spectral norm; S stays fixed.

Random draws use numpy's PCG64 (``numpy.random.default_rng(seed)``) in the
fixed order spectrum -> cluster centres -> Q's Gaussian -> L's Gaussian; the
optional torch path does the dense algebra on a device but draws the same
numbers on the host first.
"""
from __future__ import annotations

import math

import numpy as np

LOW_FRACTION = 0.2
N_CLUSTERS = 5
CLUSTER_SIZE = 4
CLUSTER_WIDTH = 1e-3
L_OFFDIAG = 0.05


def _cgauss(rng, shape):
    """Complex Gaussian with E|z|^2 = 1 (real and imaginary parts N(0, 1/2))."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * math.sqrt(0.5)


def spectrum(n: int, rng) -> np.ndarray:
    """Eigenvalues of the synthetic standard-form matrix, ascending."""
    n_low = int(round(LOW_FRACTION * n))
    low = rng.uniform(-1.0, 0.5, size=n_low)
    n_cl = min(N_CLUSTERS, n_low // CLUSTER_SIZE)
    half = CLUSTER_WIDTH / 2
    centres = rng.uniform(-1.0 + half, 0.5 - half, size=n_cl)
    offs = np.linspace(-half, half, CLUSTER_SIZE)
    for c in range(n_cl):
        low[c * CLUSTER_SIZE:(c + 1) * CLUSTER_SIZE] = centres[c] + offs
    high = np.exp(rng.uniform(math.log(0.5), math.log(100.0), size=n - n_low))
    return np.sort(np.concatenate([low, high]))


def _herm(M):
    return (M + M.conj().T) / 2


class Problem:
    """One generalized eigenproblem H x = lam S x with known spectrum."""

    def __init__(self, H, S, L, A, Q, lam):
        self.H, self.S, self.L, self.A, self.Q, self.lam = H, S, L, A, Q, lam

    @property
    def n(self):
        return self.H.shape[0]

    def exact_X(self, nev):
        """Generalized eigenvectors L^{-H} Q[:, :nev] of the lowest nev
        eigenvalues (exact up to rounding of this construction)."""
        import scipy.linalg as sl
        idx = np.argsort(self.lam, kind="stable")[:nev]
        return sl.solve_triangular(self.L.conj().T, self.Q[:, idx], lower=False)


def make_problem(n: int, seed: int, spectrum_fn=spectrum) -> Problem:
    """A single DGEVP of the synthetic FLAPW law (numpy, host memory)."""
    rng = np.random.default_rng(seed)
    lam = spectrum_fn(n, rng)
    G = _cgauss(rng, (n, n))
    Q, R = np.linalg.qr(G)
    # fix the column phases so that Q is a deterministic function of G
    d = np.diag(R)
    Q = Q * (d / np.abs(d))[None, :]
    A = _herm((Q * lam[None, :]) @ Q.conj().T)
    Gl = _cgauss(rng, (n, n))
    L = np.eye(n, dtype=np.complex128) + L_OFFDIAG * np.tril(Gl, -1) / math.sqrt(n)
    S = _herm(L @ L.conj().T)
    H = _herm(L @ A @ L.conj().T)
    return Problem(np.asfortranarray(H), np.asfortranarray(S), np.asfortranarray(L), np.asfortranarray(A), Q, lam)


def spectral_norm_herm(M, iters=30, seed=12345):
    """||M||_2 of a Hermitian matrix by Lanczos-free power iteration (input
    construction only)."""
    rng = np.random.default_rng(seed)
    v = _cgauss(rng, (M.shape[0],))
    v /= np.linalg.norm(v)
    s = 0.0
    for _ in range(iters):
        w = M @ v
        s = np.linalg.norm(w)
        v = w / s
    return float(s)


def perturbation(n: int, rng, iters=30):
    """(E + E^H)/2 with E complex Gaussian scaled to unit spectral norm
    (||E||_2 from power iteration on E^H E)."""
    E = _cgauss(rng, (n, n))
    v = _cgauss(rng, (n,))
    v /= np.linalg.norm(v)
    s = 1.0
    for _ in range(iters):
        w = E.conj().T @ (E @ v)
        s = np.linalg.norm(w)
        v = w / s
    E /= math.sqrt(s)
    return _herm(E)


def make_sequence(n: int, steps: int, seed: int, eps: float = 1e-4):
    """Correlated sequence A_{l+1} = A_l + eps ||A_l||_2 (E + E^H)/2 with S
    fixed; yields Problem objects (lam and Q describe A_0 only; later
    problems have no closed-form spectrum)."""
    p0 = make_problem(n, seed)
    yield p0
    rng = np.random.default_rng(seed + 1_000_003)
    A = p0.A
    for _ in range(1, steps):
        nrm = spectral_norm_herm(A)
        A = _herm(A + eps * nrm * perturbation(n, rng))
        H = _herm(p0.L @ A @ p0.L.conj().T)
        yield Problem(np.asfortranarray(H), p0.S, p0.L, np.asfortranarray(A), None, None)


def make_sequence_varying_s(n: int, steps: int, seed: int, eps: float = 1e-4, eps_s: float = 1e-4):
    """As make_sequence, with the overlap matrix changing along the sequence
    too: L_{l+1} = L_l + eps_s tril(G, -1)/sqrt(n) (G complex Gaussian),
    S_l = L_l L_l^H, H_l = L_l A_l L_l^H.  L_l keeps a unit diagonal, so it is
    exactly the Cholesky factor of S_l."""
    rng = np.random.default_rng(seed + 2_000_003)
    L = None
    for ell, p in enumerate(make_sequence(n, steps, seed, eps)):
        if ell == 0:
            L = p.L
            yield p
            continue
        L = L + eps_s * np.tril(_cgauss(rng, (n, n)), -1) / math.sqrt(n)
        S = _herm(L @ L.conj().T)
        H = _herm(L @ p.A @ L.conj().T)
        yield Problem(np.asfortranarray(H), np.asfortranarray(S), np.asfortranarray(L), p.A, None, None)


# --------------------------------------------------------------------------
# Device (torch) variant for large sizes: same host draws, dense algebra on
# the device.  Tensors come back column-major (transposed storage), complex128.
# --------------------------------------------------------------------------

def _colmajor(t):
    """Return a tensor whose storage is column-major (t.mT is contiguous)."""
    return t.mT.contiguous().mT


def _cgauss_device(gen, shape, device):
    """Complex Gaussian drawn on the device from a seeded torch generator
    (E|z|^2 = 1); a faster stand-in for the host draws at large sizes."""
    import torch
    re = torch.randn(shape, generator=gen, device=device, dtype=torch.float64)
    im = torch.randn(shape, generator=gen, device=device, dtype=torch.float64)
    return torch.complex(re, im) * math.sqrt(0.5)


def make_problem_torch(n: int, seed: int, device="cuda", rng_kind: str = "host"):
    """Device variant of make_problem.  rng_kind "host" draws the Gaussian
    matrices with numpy (the same numbers as make_problem); "device" draws
    them on the device from torch generators seeded with the same seed (other
    numbers, same distribution; for the large benchmark forms)."""
    import torch
    rng = np.random.default_rng(seed)
    lam = spectrum(n, rng)
    if rng_kind == "device":
        gen = torch.Generator(device=device)
        gen.manual_seed(seed)
        draw = lambda shape: _cgauss_device(gen, shape, device)
    else:
        draw = lambda shape: torch.from_numpy(_cgauss(rng, shape)).to(device)
    G = draw((n, n))
    Q, R = torch.linalg.qr(G)
    d = torch.diagonal(R)
    Q = Q * (d / d.abs())[None, :]
    lam_t = torch.from_numpy(lam).to(device=device, dtype=torch.complex128)
    A = (Q * lam_t[None, :]) @ Q.conj().T
    A = (A + A.conj().T) / 2
    Gl = draw((n, n))
    L = torch.eye(n, dtype=torch.complex128, device=device) + L_OFFDIAG * torch.tril(Gl, -1) / math.sqrt(n)
    S = L @ L.conj().T
    S = (S + S.conj().T) / 2
    H = L @ A @ L.conj().T
    H = (H + H.conj().T) / 2
    del G, R, Gl
    return {"H": _colmajor(H), "S": _colmajor(S), "L": L, "A": A, "Q": Q, "lam": lam}


def make_sequence_torch(n: int, steps: int, seed: int, eps: float = 1e-4, device="cuda", eps_decay: float = 1.0,
                        rng_kind: str = "host"):
    """Device variant of make_sequence; yields dicts with H (and S, L for the
    first problem).  Step l (l >= 1) perturbs by eps * eps_decay**(l - 1)
    (eps_decay < 1: a converging self-consistent cycle).  rng_kind as in
    make_problem_torch."""
    import torch
    p0 = make_problem_torch(n, seed, device, rng_kind)
    yield p0
    A, L, S0 = p0["A"], p0["L"], p0["S"]
    del p0  # keep only what the later steps need (S, L, A)
    rng = np.random.default_rng(seed + 1_000_003)
    if rng_kind == "device":
        gen = torch.Generator(device=device)
        gen.manual_seed(seed + 1_000_003)
        draw = lambda shape: _cgauss_device(gen, shape, device)
    else:
        draw = lambda shape: torch.from_numpy(_cgauss(rng, shape)).to(device)
    for step in range(1, steps):
        v = torch.from_numpy(_cgauss(np.random.default_rng(12345), (n,))).to(device)
        v = v / torch.linalg.vector_norm(v)
        s = 1.0
        for _ in range(30):
            w = A @ v
            s = torch.linalg.vector_norm(w)
            v = w / s
        nrm = float(s)
        E = draw((n, n))
        u = draw((n,))
        u = u / torch.linalg.vector_norm(u)
        se = 1.0
        for _ in range(30):
            w = E.conj().T @ (E @ u)
            se = torch.linalg.vector_norm(w)
            u = w / se
        E = E / math.sqrt(float(se))
        P = (E + E.conj().T) / 2
        A = A + eps * eps_decay ** (step - 1) * nrm * P
        A = (A + A.conj().T) / 2
        H = L @ A @ L.conj().T
        H = (H + H.conj().T) / 2
        del E, P
        yield {"H": _colmajor(H), "S": S0, "L": L, "A": A}
