"""The batch solver: many independent problems of different sizes solved in
lockstep, their filters' degree steps run as grouped launches (optionally
replayed from a captured HIP graph), the grouped tile shape chosen online.

Every member must meet the same acceptance bar as a single solve (the
oracle's eigenvalues for the small configuration, the exact spectrum and the
1e-10 generalized residual for the others); graph replay must give the same
bits as eager launches; a failing member must not disturb the others."""
import numpy as np
import pytest
import scipy.linalg as sl

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


def _check(p, ev, X, nev, tol=1e-10):
    """Eigenvalues against the constructed spectrum (or, for a perturbed
    member of a sequence, a dense library solver); generalized residuals."""
    hn = _checks.spectral_norm(p.H)
    lam = np.sort(p.lam) if p.lam is not None else sl.eigh(p.H, p.S, eigvals_only=True)
    ok, dmax = _checks.eig_ok(ev, lam[:nev], hn)
    assert ok, dmax
    r = _checks.gen_residuals(p.H, p.S, X, ev)
    assert r.max() <= tol * hn, r.max() / hn


def _nev(n):
    return max(4, n // 10), max(2, n // 50)


def test_batch_cold_members_match_oracle_and_spectrum(lib):
    """Three cold problems (the small configuration n=512 among them) in one
    batch; online tile choice and graph replay on."""
    probs = [workloads.make_problem(512, 0), workloads.make_problem(333, 41), workloads.make_problem(200, 7)]
    nevs = [51, 33, 20]
    nexs = [13, 7, 5]
    b = lib.Batch([p.n for p in probs], use_graph=True, degree=10, seed=0)
    ev, X, infos, st, rep = b.solve([_t(p.H) for p in probs], [_t(p.S) for p in probs], nevs, nexs, tol=1e-10)
    assert st == [0, 0, 0]
    assert rep["converged_members"] == 3
    ref = oracle.solve(probs[0].H, probs[0].S, 51, 13, tol=1e-10, degree=10, seed=0)
    assert np.abs(ev[0] - ref["evals"]).max() <= 1e-10
    for i, p in enumerate(probs):
        _check(p, ev[i], _np(X[i]), nevs[i])
        assert infos[i]["converged"] >= nevs[i]
        assert infos[i]["filter_flops"] > 0
    # online choice: six candidate shapes tried, the fastest kept, or a
    # narrower one within 2 % of it
    assert rep["outer_iterations"] >= 6
    assert rep["tile_config"] in (3, 4, 5, 7, 11, 12)
    rates = rep["tile_rate"]
    assert len(rates) == 16
    tried = [c for c in (3, 4, 5, 7, 11, 12) if rates[c] > 0]
    assert len(tried) == 6
    width = {3: 64, 4: 64, 5: 128, 7: 32, 11: 64, 12: 80}
    top = max(tried, key=lambda c: rates[c])
    chosen = rep["tile_config"]
    assert chosen == top or (rates[chosen] >= 0.98 * rates[top] and width[chosen] < width[top])
    assert all(not (width[c] < width[chosen] and rates[c] >= 0.98 * rates[top]) for c in tried)
    assert rep["graph"] == 1
    assert rep["grouped_launches"] == 10 * rep["outer_iterations"]
    assert rep["filter_flops"] == pytest.approx(sum(i["filter_flops"] for i in infos), rel=1e-12)
    b.close()


@pytest.mark.parametrize("tile,precision", [(3, 0), (11, 0), (12, 0), (12, 2)])
def test_batch_graph_replay_equals_eager_along_sequences(lib, tile, precision):
    """Three sequences of three correlated problems each (S fixed, warm
    starts).  With a pinned tile shape (64 x 64 x 8; 64 x 64 x 16 with eight
    waves; 64 x 80 x 16) the captured graph and the eager launches must
    produce identical bits at every step (each iteration replays the graph
    with the members' own eager work in between); in FP64 and with the FP32
    filter on the Ritz residual (whose grouped steps carry the forcing term
    and skip the first product)."""
    sizes = [260, 180, 300]
    seqs = [list(workloads.make_sequence(n, 3, 70 + i)) for i, n in enumerate(sizes)]
    out = {}
    for use_graph in (False, True):
        b = lib.Batch(sizes, use_graph=use_graph, degree=10, seed=2, filter_tile=tile, precision=precision)
        res = []
        for ell in range(3):
            H = [_t(s[ell].H) for s in seqs]
            S = [_t(s[ell].S) if ell == 0 else None for s in seqs]
            nev = [_nev(n)[0] for n in sizes]
            nex = [_nev(n)[1] for n in sizes]
            ev, X, infos, st, rep = b.solve(H, S, nev, nex, tol=1e-10)
            assert st == [0, 0, 0]
            assert rep["graph"] == (1 if use_graph else 0)
            assert rep["tile_config"] == tile
            for i in range(3):
                assert infos[i]["warm_start"] == (1 if ell > 0 else 0)
                assert (infos[i]["iterations_fp32"] == infos[i]["iterations"]) == (precision == 2)
                _check(seqs[i][ell], ev[i], _np(X[i]), nev[i])
            res.append(([e.copy() for e in ev], [_np(x) for x in X], [i["iterations"] for i in infos]))
        out[use_graph] = res
        b.close()
    for ell in range(3):
        e0, x0, it0 = out[False][ell]
        e1, x1, it1 = out[True][ell]
        assert it0 == it1
        for i in range(3):
            assert np.array_equal(e0[i], e1[i])
            assert np.array_equal(x0[i], x1[i])


@pytest.mark.parametrize("precision", [1, 2])
def test_batch_mixed_precision_reaches_fp64_tolerance(lib, precision):
    probs = [workloads.make_problem(400, 3), workloads.make_problem(256, 9)]
    nevs, nexs = [40, 26], [8, 6]
    b = lib.Batch([p.n for p in probs], use_graph=True, degree=10, seed=0, precision=precision)
    ev, X, infos, st, rep = b.solve([_t(p.H) for p in probs], [_t(p.S) for p in probs], nevs, nexs, tol=1e-10)
    assert st == [0, 0]
    for i, p in enumerate(probs):
        assert infos[i]["iterations_fp32"] > 0
        if precision == 2:
            assert infos[i]["iterations_fp32"] == infos[i]["iterations"]
            assert infos[i]["filter_launches_fp32"] == infos[i]["filter_launches"]
        _check(p, ev[i], _np(X[i]), nevs[i])
    b.close()


def test_batch_failing_member_leaves_others_intact(lib):
    """Member 1's S is not positive definite: it reports CHFSI_ENOTPD, the
    call returns that status, and the other members still converge."""
    import torch
    probs = [workloads.make_problem(200, 1), workloads.make_problem(150, 2), workloads.make_problem(180, 3)]
    S = [_t(p.S) for p in probs]
    S[1] = -torch.eye(150, dtype=torch.complex128, device="cuda")
    b = lib.Batch([p.n for p in probs], use_graph=False, degree=10, seed=0)
    ev, X, infos, st, rep = b.solve([_t(p.H) for p in probs], S, [20, 15, 18], [4, 3, 4], tol=1e-10,
                                    raise_on_error=False)
    assert st == [0, -2, 0]
    assert rep["converged_members"] == 2
    for i in (0, 2):
        _check(probs[i], ev[i], _np(X[i]), [20, 15, 18][i])
    b.close()


def test_batch_rejects_bad_arguments(lib):
    b = lib.Batch([64, 80], use_graph=False, degree=8)
    p0, p1 = workloads.make_problem(64, 0), workloads.make_problem(80, 1)
    with pytest.raises(lib.ChfsiError) as e:
        b.solve([_t(p0.H), _t(p1.H)], [_t(p0.S), _t(p1.S)], [10, 90], [2, 2], tol=1e-10)
    assert e.value.status == -1
    with pytest.raises(lib.ChfsiError) as e:
        b.solve([_t(p0.H), _t(p1.H)], [_t(p0.S), _t(p1.S)], [10, 10], [2, 0], tol=1e-10)  # no extra column
    assert e.value.status == -1
    with pytest.raises(ValueError):
        b.solve([_t(p0.H)], [_t(p0.S)], [10], [2])
    with pytest.raises(lib.ChfsiError):
        lib.Batch([64], filter_tile=6)  # not a grouped tile shape
    b.close()


def test_batch_members_at_configuration_sizes(lib):
    """Four k-point sequences with n drawn like the batching configuration's
    (uniform in [2000, 6000]; nev = n/10, nex = nev/10), two steps each, mixed
    precision, graph replay on: every member's eigenvalues against a library
    eigensolver (rocSOLVER through torch) on its step's standard-form matrix,
    and its generalized residuals, at both steps.  Gaussian draws on the
    device."""
    import torch
    sizes = [int(v) for v in np.random.default_rng(3).integers(2000, 6001, 4)]
    nevs = [n // 10 for n in sizes]
    nexs = [max(1, v // 10) for v in nevs]
    gens = [workloads.make_sequence_torch(n, 2, 3 + i, device="cuda", rng_kind="device") for i, n in enumerate(sizes)]
    b = lib.Batch(sizes, use_graph=True, degree=20, seed=0, precision=1)
    S0 = None
    for ell in range(2):
        ps = [next(g) for g in gens]
        if ell == 0:
            S0 = [p["S"] for p in ps]
        ev, X, infos, st, rep = b.solve([p["H"] for p in ps], S0 if ell == 0 else [None] * 4, nevs, nexs, tol=1e-10)
        assert st == [0, 0, 0, 0]
        for i, p in enumerate(ps):
            ref = torch.linalg.eigvalsh(p["A"]).cpu().numpy()[:nevs[i]]
            hn = float(np.abs(torch.linalg.eigvalsh(p["H"]).cpu().numpy()).max())
            ok, dmax = _checks.eig_ok(ev[i], ref, hn)
            assert ok, (ell, i, dmax)
            lt = torch.from_numpy(ev[i]).cuda().to(torch.complex128)
            R = p["H"] @ X[i] - (S0[i] @ X[i]) * lt[None, :]
            assert float(torch.linalg.vector_norm(R, dim=0).max()) <= 1e-10 * hn
            assert infos[i]["warm_start"] == (1 if ell > 0 else 0)
        del X, ps
    assert rep["graph"] == 1
    b.close()
