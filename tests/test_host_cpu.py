"""Host-side logic on the CPU: the correlation angle of the warm/cold study
(Sec. 2), the binding's argument marshalling, and the benchmark's report
helpers.  No GPU and no compute through the library."""
import math

import numpy as np
import pytest
import torch

import bench
from paper_1305_5120_amd import chfsi


def _spd(n, rng):
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    L = np.eye(n) + 0.1 * np.tril(G, -1) / math.sqrt(n)
    return L @ L.conj().T


def _s_orthonormal_pair(n, theta, rng, S):
    """x, y with <x, x>_S = <y, y>_S = 1 and angle theta in the S inner
    product: y = cos(theta) x + sin(theta) z, z S-orthogonal to x."""
    def snorm(v):
        return math.sqrt(float(np.real(v.conj() @ S @ v)))
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x /= snorm(x)
    z = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    z -= x * (x.conj() @ S @ z)
    z /= snorm(z)
    return x, math.cos(theta) * x + math.sin(theta) * z


@pytest.mark.parametrize("theta", [1e-10, 1e-6, 1e-3, 0.1, 0.7, 1.5])
def test_theta_against_direct_arccos_and_construction(theta):
    rng = np.random.default_rng(int(theta * 1e6) + 3)
    n = 40
    S = _spd(n, rng)
    x, y = _s_orthonormal_pair(n, theta, rng, S)
    # a phase on the new vector does not change the angle
    y = y * np.exp(1j * 0.37)
    got = bench.theta_angles(torch.from_numpy(x[:, None]), torch.from_numpy(y[:, None]), torch.from_numpy(S))
    assert got.shape == (1,)
    assert abs(got[0] - theta) <= 1e-12 + 1e-9 * theta, (got[0], theta)
    if theta >= 1e-3:
        direct = math.acos(min(1.0, abs(complex(x.conj() @ S @ y))))
        assert abs(got[0] - direct) <= 1e-9 * max(1.0, theta)


def test_theta_columnwise():
    rng = np.random.default_rng(5)
    n = 30
    S = _spd(n, rng)
    thetas = [0.01, 0.2, 1e-7]
    pairs = [_s_orthonormal_pair(n, t, rng, S) for t in thetas]
    X0 = torch.from_numpy(np.stack([p[0] for p in pairs], axis=1))
    X1 = torch.from_numpy(np.stack([p[1] for p in pairs], axis=1))
    got = bench.theta_angles(X0, X1, torch.from_numpy(S))
    assert np.allclose(got, thetas, rtol=1e-8, atol=1e-13)


def test_colmajor_materialises_conjugate_and_negative_views():
    a = torch.randn(5, 4, dtype=torch.complex128)
    for view in (a.conj(), a.T.conj().T, -a.conj()):
        c, ld = chfsi.colmajor(view)
        assert not c.is_conj() and not c.is_neg()
        assert torch.equal(c, view.resolve_conj().resolve_neg())
        # the storage the pointer names is column-major with leading dim ld
        assert c.stride(0) == 1 and ld >= 5
        flat = torch.as_strided(c, (5, 4), (1, ld))
        assert torch.equal(flat, view.resolve_conj().resolve_neg())


def test_colmajor_row_major_input_is_not_read_transposed():
    a = torch.arange(12, dtype=torch.float64).reshape(3, 4).to(torch.complex128)
    c, ld = chfsi.colmajor(a)
    assert ld == 3 and c.stride(0) == 1
    assert torch.equal(c, a)


def test_shape_checks_reject_wrong_sizes():
    t = torch.zeros(6, 5, dtype=torch.complex128)
    chfsi._check_shape(t, 6, 5, "H")
    for rows, cols in ((5, 5), (6, 6), (7, 5)):
        with pytest.raises(ValueError):
            chfsi._check_shape(t, rows, cols, "H")
    # a view into a larger matrix has the view's shape
    big = torch.zeros(10, 10, dtype=torch.complex128)
    with pytest.raises(ValueError):
        chfsi._check_shape(big[:6, :6], 10, 10, "H")


def test_device_checks_reject_host_and_wrong_dtype():
    with pytest.raises(TypeError):
        chfsi._check_dev(torch.zeros(4, 4, dtype=torch.complex128), "H")  # host tensor
    with pytest.raises(TypeError):
        chfsi._check_dev(np.zeros((4, 4)), "H")


def test_eigenpair_report():
    lam = np.array([3.0, -1.0, 0.5, 7.0])
    ev64 = np.array([-1.0 + 1e-14, 0.5, 3.0])
    evm = np.array([-1.0, 0.5 + 2e-13, 3.0])
    evr = np.array([-1.0, 0.5, 3.0 - 3e-13])
    r = bench._eig_report(lam, ev64, {"mixed": evm, "ritz32": evr}, 7.0)
    assert len(r["fp64_vs_exact"]) == 3
    assert r["max"]["fp64_vs_exact"] == pytest.approx(1e-14 / 7.0, rel=1e-2)
    assert r["max"]["mixed_vs_exact"] == pytest.approx(2e-13 / 7.0, rel=1e-2)
    assert r["mixed_vs_fp64"][0] == pytest.approx(1e-14 / 7.0, rel=1e-2)
    assert r["max"]["ritz32_vs_exact"] == pytest.approx(3e-13 / 7.0, rel=1e-2)
    assert r["ritz32_vs_fp64"][2] == pytest.approx(3e-13 / 7.0, rel=1e-2)


def test_bench_refuses_several_gpus(capsys):
    import subprocess
    import sys
    import os
    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(bench.__file__), "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The C oracle built with -fsanitize=address,undefined (host code, gcc)
    runs its solve's paths (cold, warm with bounds, iteration limit, S not
    positive definite, invalid sizes) with no sanitizer report, and the cold
    solve finds the constructed smallest eigenvalues."""
    import os
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    here = os.path.dirname(os.path.abspath(__file__))
    root = os.path.dirname(here)
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-D_POSIX_C_SOURCE=200809L", "-o", exe,
           os.path.join(here, "oracle_sanitize_main.c"), os.path.join(root, "oracle", "chfsi_oracle.c"), "-lm"]
    b = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert b.returncode == 0, b.stdout
    # (verify_asan_link_order=0: a library preloaded by the environment may
    # come before the sanitizer runtime in the load order)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=120)
    assert r.returncode == 0 and "oracle sanitizer run ok" in r.stdout, r.stdout


def test_low_precision_roofline_takes_the_operand_peak():
    r2 = bench.low_precision_roofline(2, 2.0e14, 1.5)
    r3 = bench.low_precision_roofline(3, 2.0e14, 0.4)
    assert r2["peak"] == 157.3 and r2["operands"] == "fp32"
    assert r3["peak"] == 2500.0 and r3["operands"] == "fp16"
    assert r3["achieved"] == pytest.approx(500.0) and r3["frac"] == pytest.approx(0.2)
    assert bench.low_precision_roofline(1, 0.0, 0.0)["achieved"] is None
