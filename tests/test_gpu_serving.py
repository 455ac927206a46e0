"""The serving loop: many sequences, concurrent workers, resident warm state,
admission by device-memory budget.  Each result must be the same whether its
sequence runs alone or mixed with the others (deterministic kernels, one
context and stream per solve), and must meet the FP64 tolerance."""
import numpy as np
import pytest
import scipy.linalg as sl

import workloads
from tests import _checks

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    a = np.asarray(a, dtype=np.complex128)
    return torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda").mT


SIZES = {0: 150, 1: 220, 2: 260, 3: 300}
STEPS = 3


@pytest.fixture(scope="module")
def sequences(gpu):
    out = {}
    for s, n in SIZES.items():
        seq = list(workloads.make_sequence(n, STEPS, 500 + s))
        out[s] = [(p, _t(p.H), _t(p.S)) for p in seq]
    return out


def _nev(n):
    return max(4, n // 12), max(2, n // 60)


def _run(lib, sequences, order, workers):
    srv = lib.Server(workers=workers, hbm_budget_bytes=8 << 30, degree=10, seed=0)
    tickets = {}
    for s, ell in order:
        p, H, S = sequences[s][ell]
        nev, nex = _nev(p.n)
        tickets[(s, ell)] = srv.submit(s, H, S, nev, nex, tol=1e-10)
    res = {}
    for key, t in tickets.items():
        ev, X, info, lat, st = srv.wait(t)
        assert st == 0
        res[key] = (ev, X.cpu().numpy(), info)
    stats = srv.stats()
    srv.close()
    return res, stats


def test_server_results_same_alone_and_in_the_mix(lib, sequences):
    alone = {}
    for s in SIZES:
        r, _ = _run(lib, sequences, [(s, ell) for ell in range(STEPS)], workers=1)
        alone.update(r)
    mix_order = [(s, ell) for ell in range(STEPS) for s in SIZES]
    mixed, stats = _run(lib, sequences, mix_order, workers=3)
    assert stats["completed"] == len(mix_order) and stats["failed"] == 0
    assert stats["p99_latency"] >= stats["p50_latency"] > 0
    for key in alone:
        ev_a, X_a, info_a = alone[key]
        ev_m, X_m, info_m = mixed[key]
        # same arithmetic: identical to the last bit
        assert np.array_equal(ev_a, ev_m), key
        assert np.array_equal(X_a, X_m), key
        s, ell = key
        p = sequences[s][ell][0]
        nev = len(ev_a)
        hn = _checks.spectral_norm(p.H)
        ref = sl.eigh(p.H, p.S, eigvals_only=True)[:nev]
        assert _checks.eig_ok(ev_a, ref, hn)[0]
        r = _checks.gen_residuals(p.H, p.S, X_a, ev_a)
        assert r.max() <= 1e-10 * hn
        assert info_a["warm_start"] == (1 if ell > 0 else 0)


def test_server_admits_within_budget(lib, sequences):
    # room for about one context at a time: requests are serialized, peak
    # memory stays under the budget, every request still completes
    p, H, S = sequences[3][0]
    budget = 60 * 300 * 300 * 16
    srv = lib.Server(workers=3, hbm_budget_bytes=budget, degree=10)
    tickets = [srv.submit(s, *sequences[s][0][1:], *_nev(sequences[s][0][0].n)) for s in SIZES]
    for t in tickets:
        ev, X, info, lat, st = srv.wait(t)
        assert st == 0
    st = srv.stats()
    assert st["peak_bytes"] <= budget and st["completed"] == len(SIZES)
    srv.close()


def test_server_rejects_request_larger_than_budget(lib, sequences):
    p, H, S = sequences[0][0]
    srv = lib.Server(workers=2, hbm_budget_bytes=1 << 20, degree=10)
    t = srv.submit(0, H, S, *_nev(p.n))
    ev, X, info, lat, st = srv.wait(t, raise_on_error=False)
    assert st == -5
    srv.close()


def test_server_rejects_invalid_block_sizes(lib, sequences):
    """nev + nex above n, and no extra column while the block is not the
    whole space, are refused at submission."""
    p, H, S = sequences[0][0]
    srv = lib.Server(workers=1, degree=10)
    for nev, nex in ((p.n, 1), (10, 0)):
        with pytest.raises(lib.ChfsiError) as e:
            srv.submit(0, H, S, nev, nex)
        assert e.value.status == -1
    srv.close()


@pytest.mark.parametrize("precision", [1, 2, 3])
def test_server_at_configuration_sizes(lib, precision):
    """Three sequences with n in the serving configuration's range (2000,
    4500, 8000; nev 3 %, 10 % and 5 % of n, nex = nev/10), two steps each,
    both mixed-precision forms, two workers under the 200 GB budget, submitted
    interleaved: every result against a library eigensolver (rocSOLVER
    through torch) on its step's standard-form matrix, with generalized
    residuals.  Gaussian draws on the device."""
    import torch
    cases = [(2000, 0.03), (4500, 0.10), (8000, 0.05)]
    seqs = [list(workloads.make_sequence_torch(n, 2, 700 + i, device="cuda", rng_kind="device"))
            for i, (n, _) in enumerate(cases)]
    srv = lib.Server(workers=2, hbm_budget_bytes=200 << 30, degree=20, seed=0, precision=precision)
    tickets = {}
    for ell in range(2):
        for s, (n, f) in enumerate(cases):
            nev = int(n * f)
            p = seqs[s][ell]
            tickets[(s, ell)] = srv.submit(s, p["H"], seqs[s][0]["S"], nev, max(1, nev // 10), tol=1e-10)
    for (s, ell), t in tickets.items():
        ev, X, info, lat, st = srv.wait(t)
        assert st == 0, (s, ell)
        p = seqs[s][ell]
        nev = len(ev)
        ref = torch.linalg.eigvalsh(p["A"]).cpu().numpy()[:nev]
        hn = float(np.abs(torch.linalg.eigvalsh(p["H"]).cpu().numpy()).max())
        ok, dmax = _checks.eig_ok(ev, ref, hn)
        assert ok, (s, ell, dmax)
        lt = torch.from_numpy(ev).cuda().to(torch.complex128)
        R = p["H"] @ X - (seqs[s][0]["S"] @ X) * lt[None, :]
        assert float(torch.linalg.vector_norm(R, dim=0).max()) <= 1e-10 * hn
        del X, R
    stats = srv.stats()
    assert stats["completed"] == 6 and stats["failed"] == 0
    srv.close()


def test_server_reuses_the_overlap_factor(lib, sequences):
    """Requests that pass S = None (the sequence's overlap matrix unchanged)
    reuse the factor a worker holds, or factor the remembered matrix again:
    the same bits as passing S every time, with one worker (always the
    holder) and with three (the holder when idle, else a new factorization)."""
    order = [(s, ell) for ell in range(STEPS) for s in SIZES]
    ref, _ = _run(lib, sequences, order, workers=1)
    for workers in (1, 3):
        srv = lib.Server(workers=workers, hbm_budget_bytes=8 << 30, degree=10, seed=0)
        tickets = {}
        for s, ell in order:
            p, H, S = sequences[s][ell]
            nev, nex = _nev(p.n)
            tickets[(s, ell)] = srv.submit(s, H, S if ell == 0 else None, nev, nex, tol=1e-10)
        for key, t in tickets.items():
            ev, X, info, lat, st = srv.wait(t)
            assert st == 0, key
            assert np.array_equal(ev, ref[key][0]), (workers, key)
            assert np.array_equal(X.cpu().numpy(), ref[key][1]), (workers, key)
        srv.close()


def test_server_request_without_any_overlap_matrix_fails(lib, sequences):
    p, H, S = sequences[0][0]
    srv = lib.Server(workers=1, degree=10)
    t = srv.submit(7, H, None, *_nev(p.n))
    ev, X, info, lat, st = srv.wait(t, raise_on_error=False)
    assert st == -1
    srv.close()


def test_server_context_reused_across_sizes(lib):
    """One worker takes a large problem, then smaller and larger ones: its
    context serves every size from the same buffers (growing for the larger
    one), and each result is the same bits as on a fresh server (the split
    choices do not depend on the sizes served before).  Sizes above 1024
    rows take the split-K products."""
    import torch
    cases = [(2100, 30), (1100, 20), (2400, 24), (1100, 20)]
    probs = [workloads.make_problem_torch(n, 900 + i, device="cuda", rng_kind="device") for i, (n, _) in
             enumerate(cases)]
    fresh = []
    for (n, nev), p in zip(cases, probs):
        srv = lib.Server(workers=1, hbm_budget_bytes=64 << 30, degree=10, seed=0)
        ev, X, info, lat, st = srv.wait(srv.submit(0, p["H"], p["S"], nev, 12, tol=1e-10))
        assert st == 0
        fresh.append((ev, X.cpu().numpy()))
        srv.close()
    srv = lib.Server(workers=1, hbm_budget_bytes=64 << 30, degree=10, seed=0)
    tickets = [srv.submit(i, p["H"], p["S"], nev, 12, tol=1e-10) for i, ((n, nev), p) in enumerate(zip(cases, probs))]
    for i, t in enumerate(tickets):
        ev, X, info, lat, st = srv.wait(t)
        assert st == 0
        assert np.array_equal(ev, fresh[i][0]), i
        assert np.array_equal(X.cpu().numpy(), fresh[i][1]), i
        ok, dmax = _checks.eig_ok(ev, np.sort(probs[i]["lam"])[:cases[i][1]],
                                  float(torch.linalg.eigvalsh(probs[i]["H"]).abs().max()))
        assert ok, (i, dmax)
    srv.close()
