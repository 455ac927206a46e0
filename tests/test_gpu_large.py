"""The serving configuration's largest sizes (Sec. 2 sequences; Table 1's
problems extended to n = 20000, nev up to 20 % of n): the reduced
eigensolver at the widest block, k = 4400, and problems with n = 20000 -
through the server (nev = 3 %, cold) and through a context (nev = 20 %,
warm-started from the constructed eigenvectors perturbed by 1e-8, so that a
few outer iterations at the full width suffice).  Gaussian draws on the
device; references are the spectrum known by construction and a library
eigensolver (rocSOLVER through torch)."""
import numpy as np
import pytest

import workloads
from tests import _checks

pytestmark = pytest.mark.gpu

N_TOP = 20000


def _hnorm(H):
    import torch
    v = torch.ones(H.shape[0], dtype=torch.complex128, device=H.device)
    for _ in range(50):
        v = H @ v
        v = v / torch.linalg.vector_norm(v)
    return float(torch.linalg.vector_norm(H @ v))


def _residual_max(H, S, X, ev):
    import torch
    lt = torch.from_numpy(np.asarray(ev)).to(device=X.device, dtype=torch.complex128)
    worst = 0.0
    for c0 in range(0, X.shape[1], 1000):  # column chunks bound the temporaries
        Xc = X[:, c0:c0 + 1000]
        R = H @ Xc - (S @ Xc) * lt[None, c0:c0 + 1000]
        worst = max(worst, float(torch.linalg.vector_norm(R, dim=0).max()))
        del R
    return worst


def test_eigh_widest_block_of_the_serving_configuration(lib):
    """k = 4400 (nev = 20 % of n = 20000 plus nex = nev/10): a dense complex
    Gaussian Hermitian matrix, eigenvalues against the library eigensolver,
    eigenpairs by their residual and the eigenvectors' orthonormality.  The
    orthonormality bound scales with k: every entry of Z^H Z is an inner
    product of length k, formed from vectors that many rotations and
    refinement products of length k have touched (1e-15 k = 4.4e-12)."""
    import torch
    k = 4400
    g = torch.Generator(device="cuda").manual_seed(4400)
    M = torch.complex(torch.randn(k, k, generator=g, device="cuda", dtype=torch.float64),
                      torch.randn(k, k, generator=g, device="cuda", dtype=torch.float64))
    G = ((M + M.mH) / 2).mT.contiguous().mT
    del M
    ctx = lib.create(k)
    print(f"eigh k={k}", flush=True)
    w, Z = lib.eigh(ctx, G)
    ref = torch.linalg.eigvalsh(G).cpu().numpy()
    gn = float(torch.linalg.matrix_norm(G))
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - ref).max() <= 1e-13 * gn
    wt = torch.from_numpy(w).to(device="cuda", dtype=torch.complex128)
    assert float((G @ Z - Z * wt[None, :]).abs().max()) <= 1e-12 * gn
    ctx.release()
    assert float((Z.mH @ Z - torch.eye(k, dtype=torch.complex128, device="cuda")).abs().max()) <= 1e-15 * k


@pytest.fixture(scope="module")
def top_problem(gpu):
    p = workloads.make_problem_torch(N_TOP, 4, device="cuda", rng_kind="device")
    p["hnorm"] = _hnorm(p["H"])
    yield p
    del p


def test_server_request_at_the_largest_size(lib, top_problem):
    """One cold request with n = 20000, nev = 3 % of n (600), nex = 60,
    mixed precision, admitted under the 200 GB budget: every eigenvalue
    against the constructed spectrum, the generalized residuals."""
    p = top_problem
    nev, nex = 600, 60
    srv = lib.Server(workers=1, hbm_budget_bytes=200 << 30, degree=20, seed=0, precision=1)
    print(f"server request n={N_TOP} nev={nev}", flush=True)
    t = srv.submit(0, p["H"], p["S"], nev, nex, tol=1e-10)
    ev, X, info, lat, st = srv.wait(t)
    assert st == 0
    stats = srv.stats()
    assert stats["completed"] == 1 and stats["peak_bytes"] <= 200 << 30
    srv.close()
    ok, dmax = _checks.eig_ok(ev, np.sort(p["lam"])[:nev], p["hnorm"])
    assert ok, dmax
    assert _residual_max(p["H"], p["S"], X, ev) <= 1e-10 * p["hnorm"]


def test_solve_widest_block_at_the_largest_size(lib, top_problem):
    """n = 20000, nev = 20 % of n (4000), nex = 400: the block spans the whole
    low part of the spectrum and the first values of the log-uniform part.
    Warm-started from the constructed generalized eigenvectors L^{-H} Q_k
    perturbed by 1e-8 (relative, per column): every eigenvalue against the
    constructed spectrum, the generalized residuals."""
    import torch
    p = top_problem
    nev, nex = 4000, 400
    k = nev + nex
    # X = L^{-H} Q_k from L^H X = Q_k, L^H = I + N^H with N = L - I strictly
    # lower and ||N|| about 0.05: the fixed-point iteration X <- Q_k - N^H X
    # converges geometrically (the library triangular solve runs out of
    # workspace at this size)
    NH = (p["L"] - torch.eye(N_TOP, dtype=torch.complex128, device="cuda")).mH.contiguous()
    Qk = p["Q"][:, :k].contiguous()
    Xw = Qk.clone()
    for _ in range(60):
        Xn = Qk - NH @ Xw
        done = float(torch.linalg.matrix_norm(Xn - Xw)) <= 1e-15 * float(torch.linalg.matrix_norm(Xn))
        Xw = Xn
        if done:
            break
    assert float(torch.linalg.matrix_norm(Xw + NH @ Xw - Qk)) <= 1e-13 * float(torch.linalg.matrix_norm(Qk))
    del NH, Qk, Xn
    g = torch.Generator(device="cuda").manual_seed(5)
    E = torch.complex(torch.randn(N_TOP, k, generator=g, device="cuda", dtype=torch.float64),
                      torch.randn(N_TOP, k, generator=g, device="cuda", dtype=torch.float64))
    Xw = Xw + 1e-8 * E * (torch.linalg.vector_norm(Xw, dim=0) / torch.linalg.vector_norm(E, dim=0))[None, :]
    Xw = Xw.mT.contiguous().mT
    del E
    ctx = lib.create(N_TOP, degree=20, seed=0)
    print(f"solve n={N_TOP} nev={nev} warm", flush=True)
    ev, X, info, st = lib.solve(ctx, p["H"], p["S"], nev, nex, V_warm=Xw, tol=1e-10)
    assert st == 0 and info["warm_start"] == 1
    print(f"iterations {info['iterations']}, {info['t_total']:.1f} s", flush=True)
    del Xw
    ok, dmax = _checks.eig_ok(ev, np.sort(p["lam"])[:nev], p["hnorm"])
    assert ok, dmax
    assert _residual_max(p["H"], p["S"], X, ev) <= 1e-10 * p["hnorm"]
    ctx.release()
