"""Warm-started solves (Sec. 2: each problem of a sequence starts from the
previous one's eigenvectors; Alg. 1 takes them as its input block) against
the CPU oracle run on the same warm-start path.

Sizes follow the small configuration (n = 512, nev = 51, nex = 13, degree
10, tol 1e-10) over 3-step correlated sequences.  The oracle and the library
each run their own chain: step l of the oracle starts from the oracle's step
l - 1 (its final standard-form block, carried through the generalized space,
and its filter bounds), step l of the library from the library's.  Compared
per step:
  * eigenvalues: library vs oracle element by element, |dlam| <= 1e-10 |lam|
    or <= 1e-12 ||H||_2, and both against a dense library eigensolver;
  * eigenvectors: residuals <= 1e-10 ||H||_2, S-orthonormality, and subspace
    angles per cluster-closed group against the dense solver's vectors
    (Davis-Kahan reading of the 1e-8 angle rule);
  * the start: the library reports a warm start, and its iteration count
    stays within a few of the oracle's (the paper fixes no trajectory; both
    runs take the same steps up to rounding).
Paths: the context's kept block with S cached, the kept block with a new S
(remapped through the generalized space), explicit generalized vectors on a
context that already solved another problem, chfsi_reduce with a new S
between solves, a failed reduction, a server request resumed from its
sequence's resident state, and a batch member.
"""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle
import workloads
from tests import _checks

pytestmark = pytest.mark.gpu

N, NEV, NEX, M, TOL = 512, 51, 13, 10, 1e-10


def _t(a):
    import torch
    a = np.asarray(a, dtype=np.complex128)
    return torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda").mT


def _np(t):
    return t.detach().cpu().numpy()


def _dense(p):
    """Standard form, its eigenvalues and eigenvectors from LAPACK (an
    independent library check)."""
    Li = sl.solve_triangular(p.L, np.eye(p.n), lower=True)
    A = Li @ p.H @ Li.conj().T
    A = (A + A.conj().T) / 2
    lam, V = np.linalg.eigh(A)
    return A, lam, V


def _check_step(p, ev, X, ref, label):
    hn = _checks.spectral_norm(p.H)
    ok, d = _checks.eig_ok(ev, ref["evals"], hn)
    assert ok, (label, "library vs oracle", d)
    A, lam, V = _dense(p)
    for name, e, Xs in (("library", ev, X), ("oracle", ref["evals"], ref["X"])):
        ok, d = _checks.eig_ok(e, lam[:NEV], hn)
        assert ok, (label, name, "vs dense", d)
        r = _checks.gen_residuals(p.H, p.S, Xs, e)
        assert r.max() <= TOL * hn, (label, name, r.max() / hn)
        assert _checks.s_orth_err(p.S, Xs) <= 1e-12, (label, name)
        ok, worst, ratio = _checks.subspace_check(_checks.standard_vectors(p.L, Xs), V, lam, A, e, NEV)
        assert ok, (label, name, worst, ratio)


def _oracle_chain(seq, warm_from_state=True):
    """The oracle's own warm chain: step l starts from step l - 1's final block
    mapped to the generalized space with that step's factor, and its
    bounds."""
    out = []
    prev = None
    for p in seq:
        if prev is None:
            r = oracle.solve(p.H, p.S, NEV, NEX, tol=TOL, degree=M, seed=0)
        else:
            pp, pr = prev
            Vw = oracle.backtransform(oracle.cholesky(pp.S)[0], pr["Y"]) if warm_from_state else pr["X"]
            bounds = [pr["info"]["a0"], pr["info"]["a"]] if warm_from_state else None
            r = oracle.solve(p.H, p.S, NEV, NEX, tol=TOL, degree=M, seed=0, V_warm=Vw, bounds=bounds)
        assert r["info"]["status"] == 0
        out.append(r)
        prev = (p, r)
    return out


def _close_iterations(it_lib, it_orc):
    assert abs(it_lib - it_orc) <= 3, (it_lib, it_orc)


@pytest.fixture(scope="module")
def fixed_s():
    seq = list(workloads.make_sequence(N, 3, 31))
    return seq, _oracle_chain(seq)


@pytest.fixture(scope="module")
def varying_s():
    seq = list(workloads.make_sequence_varying_s(N, 3, 37))
    return seq, _oracle_chain(seq)


def test_kept_block_with_cached_overlap(lib, fixed_s):
    """(i) S passed once, then NULL: the context's kept block and bounds."""
    seq, refs = fixed_s
    ctx = lib.create(N, degree=M, seed=0)
    for ell, (p, ref) in enumerate(zip(seq, refs)):
        ev, X, info, st = lib.solve(ctx, _t(p.H), _t(p.S) if ell == 0 else None, NEV, NEX, tol=TOL)
        assert st == 0 and info["warm_start"] == (1 if ell else 0)
        _check_step(p, ev, _np(X), ref, f"kept block, step {ell}")
        _close_iterations(info["iterations"], ref["info"]["iterations"])
    assert refs[2]["info"]["iterations"] < refs[0]["info"]["iterations"]


def test_kept_block_with_new_overlap(lib, varying_s):
    """(iii) a new S on a warm context: the kept block goes through the
    generalized space, X = L_old^{-H} Y, then Y0 = L_new^H X, with the kept
    bounds."""
    seq, refs = varying_s
    ctx = lib.create(N, degree=M, seed=0)
    for ell, (p, ref) in enumerate(zip(seq, refs)):
        ev, X, info, st = lib.solve(ctx, _t(p.H), _t(p.S), NEV, NEX, tol=TOL)
        assert st == 0 and info["warm_start"] == (1 if ell else 0)
        _check_step(p, ev, _np(X), ref, f"kept block, new S, step {ell}")
        _close_iterations(info["iterations"], ref["info"]["iterations"])
        assert info["b_upper"] >= np.max(np.linalg.eigvalsh(_dense(p)[0]))


def test_explicit_vectors_on_a_used_context(lib, varying_s):
    """(ii) explicit generalized vectors (nev columns, the rest of the block
    random) with a new S, on a context that has just solved another problem:
    the filter bounds come from a Rayleigh-Ritz step of the new start block,
    not from the context's previous problem."""
    seq, _ = varying_s
    r0 = oracle.solve(seq[0].H, seq[0].S, NEV, NEX, tol=TOL, degree=M, seed=0)
    ref = oracle.solve(seq[1].H, seq[1].S, NEV, NEX, tol=TOL, degree=M, seed=0, V_warm=r0["X"])
    assert ref["info"]["status"] == 0
    ctx = lib.create(N, degree=M, seed=0)
    # another problem first (its bounds stay in the context), then the first step
    other = workloads.make_problem(N, 99)
    lib.solve(ctx, _t(other.H), _t(other.S), NEV, NEX, tol=TOL)
    ev0, X0, _, _ = lib.solve(ctx, _t(seq[0].H), _t(seq[0].S), NEV, NEX, tol=TOL)
    lib.solve(ctx, _t(other.H), _t(other.S), NEV, NEX, tol=TOL)
    ev, X, info, st = lib.solve(ctx, _t(seq[1].H), _t(seq[1].S), NEV, NEX, V_warm=X0, tol=TOL)
    assert st == 0 and info["warm_start"] == 1
    _check_step(seq[1], ev, _np(X), ref, "explicit vectors")
    _close_iterations(info["iterations"], ref["info"]["iterations"])
    # the bounds of the start block: a0 <= smallest, a near the block's top
    assert info["a0"] <= ev[0] + 1e-12


def test_reduce_with_new_overlap_then_cached_solve(lib, varying_s):
    """chfsi_reduce with a new S between solves, then a solve with S = NULL:
    the kept block follows the new factor."""
    seq, refs = varying_s
    ctx = lib.create(N, degree=M, seed=0)
    lib.solve(ctx, _t(seq[0].H), _t(seq[0].S), NEV, NEX, tol=TOL)
    lib.reduce(ctx, _t(seq[1].H), _t(seq[1].S))
    ev, X, info, st = lib.solve(ctx, _t(seq[1].H), None, NEV, NEX, tol=TOL)
    assert st == 0 and info["warm_start"] == 1
    _check_step(seq[1], ev, _np(X), refs[1], "reduce, then cached solve")
    _close_iterations(info["iterations"], refs[1]["info"]["iterations"])


def test_failed_reduction_drops_the_kept_block(lib, varying_s):
    """A reduction that fails (S not positive definite) leaves no stale block:
    the next solve with a valid S starts cold and equals the oracle's cold
    solve."""
    seq, _ = varying_s
    ctx = lib.create(N, degree=M, seed=0)
    lib.solve(ctx, _t(seq[0].H), _t(seq[0].S), NEV, NEX, tol=TOL)
    bad = seq[1].S.copy()
    bad[5, 5] = -1.0
    with pytest.raises(lib.ChfsiError) as e:
        lib.solve(ctx, _t(seq[1].H), _t(bad), NEV, NEX, tol=TOL)
    assert e.value.status == -2
    with pytest.raises(lib.ChfsiError) as e:
        lib.solve(ctx, _t(seq[1].H), None, NEV, NEX, tol=TOL)  # no factor to reuse
    assert e.value.status == -1
    ref = oracle.solve(seq[1].H, seq[1].S, NEV, NEX, tol=TOL, degree=M, seed=0)
    ev, X, info, st = lib.solve(ctx, _t(seq[1].H), _t(seq[1].S), NEV, NEX, tol=TOL)
    assert st == 0 and info["warm_start"] == 0
    _check_step(seq[1], ev, _np(X), ref, "after a failed reduction")
    assert info["iterations"] == pytest.approx(ref["info"]["iterations"], abs=3)


def test_server_request_resumes_resident_state(lib, varying_s):
    """(iv) requests of one sequence through the server: each resumes the
    sequence's resident block (generalized space) and bounds."""
    seq, refs = varying_s
    srv = lib.Server(workers=2, hbm_budget_bytes=8 << 30, degree=M, seed=0)
    try:
        for ell, (p, ref) in enumerate(zip(seq, refs)):
            t = srv.submit(7, _t(p.H), _t(p.S), NEV, NEX, tol=TOL)
            ev, X, info, lat, st = srv.wait(t)
            assert st == 0 and info["warm_start"] == (1 if ell else 0)
            _check_step(p, ev, _np(X), ref, f"server, step {ell}")
            _close_iterations(info["iterations"], ref["info"]["iterations"])
    finally:
        srv.close()


def test_batch_member_warm_steps(lib, fixed_s):
    """A batch member's warm steps (grouped filter launches, kept block and
    bounds) against the oracle chain."""
    seq, refs = fixed_s
    b = lib.Batch([N], use_graph=True, degree=M, seed=0)
    try:
        for ell, (p, ref) in enumerate(zip(seq, refs)):
            evs, Xs, infos, sts, rep = b.solve([_t(p.H)], [_t(p.S) if ell == 0 else None], [NEV], [NEX], tol=TOL)
            assert sts[0] == 0 and infos[0]["warm_start"] == (1 if ell else 0)
            _check_step(p, evs[0], _np(Xs[0]), ref, f"batch, step {ell}")
            _close_iterations(infos[0]["iterations"], ref["info"]["iterations"])
    finally:
        b.close()


def test_mixed_precision_warm_steps(lib, fixed_s):
    """The mixed-precision filter on the kept-block path reaches the same FP64
    tolerance as the oracle chain (iterations not compared: the FP32 filter
    takes its own trajectory)."""
    seq, refs = fixed_s
    ctx = lib.create(N, degree=M, seed=0, precision=1)
    for ell, (p, ref) in enumerate(zip(seq, refs)):
        ev, X, info, st = lib.solve(ctx, _t(p.H), _t(p.S) if ell == 0 else None, NEV, NEX, tol=TOL)
        assert st == 0
        _check_step(p, ev, _np(X), ref, f"mixed, step {ell}")
