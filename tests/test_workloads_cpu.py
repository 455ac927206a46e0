"""Input generators (CPU): the device variants of the synthetic problems and
sequences.  The host-draw path reproduces the numpy generator; the
device-draw path (used by the full-size batching form) is reproducible from
its seed and keeps the spectrum law and the structure of the sequence."""
import numpy as np
import torch

import workloads


def test_host_draws_reproduce_the_numpy_generator():
    p = workloads.make_problem(96, 5)
    q = workloads.make_problem_torch(96, 5, device="cpu")
    hn = np.linalg.norm(p.H, 2)
    assert np.abs(q["H"].numpy() - p.H).max() <= 1e-13 * hn
    assert np.abs(q["S"].numpy() - p.S).max() <= 1e-13


def test_device_draws_are_reproducible_and_keep_the_spectrum():
    a = list(workloads.make_sequence_torch(80, 3, 9, device="cpu", rng_kind="device"))
    b = list(workloads.make_sequence_torch(80, 3, 9, device="cpu", rng_kind="device"))
    for x, y in zip(a, b):
        assert torch.equal(x["H"], y["H"])
    # other numbers than the host draws, the same constructed spectrum
    h = workloads.make_problem_torch(80, 9, device="cpu")
    assert not torch.equal(a[0]["H"], h["H"])
    lam = np.sort(workloads.make_problem(80, 9).lam)
    assert np.abs(np.linalg.eigvalsh(a[0]["A"].numpy()) - lam).max() <= 1e-12 * np.abs(lam).max()
    # S fixed along the sequence, H Hermitian, consecutive problems close
    for x in a[1:]:
        assert torch.equal(x["S"], a[0]["S"])
        H = x["H"].numpy()
        assert np.abs(H - H.conj().T).max() == 0.0
    d = np.linalg.norm(a[1]["H"].numpy() - a[0]["H"].numpy(), 2) / np.linalg.norm(a[0]["H"].numpy(), 2)
    assert 1e-6 < d < 1e-3
