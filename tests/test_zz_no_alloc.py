"""The allocation-free complex GEMM (chfsi_zgemm_static) against the
context-based chfsi_zgemm, through the C ABI.

Both entry points run the same kernels; the static one keeps its split-K
partial tiles in a fixed per-GPU array.  With the tile shape and split given
explicitly the two must agree bit for bit; with the automatic choice (which
may split differently under the fixed scratch) they agree to the product's
rounding.  Each test makes two calls in a row, the second smaller, so the
second reads a scratch that still holds the first call's partial tiles.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    a = np.asarray(a, dtype=np.complex128)
    return torch.from_numpy(np.ascontiguousarray(a.T)).to("cuda").mT


def _np(t):
    return t.detach().cpu().numpy()


def _cg(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _zeros(M, N):
    import torch
    return torch.zeros(N, M, dtype=torch.complex128, device="cuda").mT


# (opA, opB, M, N, K, tile, split, structure flags)
EXPLICIT = [
    [(0, 0, 1000, 300, 3000, 1, 4, 0), (1, 0, 500, 130, 1500, 7, 2, 0)],
    [(0, 1, 900, 900, 700, 2, 4, 16), (0, 0, 333, 77, 1200, 3, 3, 0)],
    [(0, 0, 1100, 150, 2500, 12, 4, 0), (1, 0, 600, 200, 1800, 11, 2, 0)],
]


@pytest.mark.parametrize("calls", EXPLICIT)
def test_static_gemm_explicit_tiles_bit_identical(lib, calls):
    import torch
    rng = np.random.default_rng(2024)
    ctx = lib.create(8)
    for opA, opB, M, N, K, tile, split, structure in calls:
        A = _cg(rng, (M, K) if opA == 0 else (K, M))
        B = _cg(rng, (K, N) if opB == 0 else (N, K))
        X, Z = _cg(rng, (M, N)), _cg(rng, (M, N))
        flags = structure | (tile << 8) | (split << 16)
        print(f"static gemm: op {opA}{opB} {M}x{N}x{K} tile {tile} split {split} flags {structure}", flush=True)
        Cs = lib.zgemm_static(opA, opB, _t(A), _t(B), _zeros(M, N), alpha=0.7, beta=-0.3, X=_t(X), gamma=1.9,
                              Z=_t(Z), flags=flags)
        Cc = lib.zgemm(ctx, opA, opB, _t(A), _t(B), alpha=0.7, beta=-0.3, X=_t(X), gamma=1.9, Z=_t(Z),
                       C=_zeros(M, N), flags=flags)
        torch.cuda.synchronize()
        cs, cc = _np(Cs), _np(Cc)
        opa = A if opA == 0 else A.conj().T
        opb = B if opB == 0 else B.conj().T
        ref = 0.7 * (opa @ opb) - 0.3 * X + 1.9 * Z
        if structure & 16:
            low = np.tril_indices(M)
            cs, cc, ref = cs[low], cc[low], ref[low]
        assert np.array_equal(cs, cc)
        assert _rel(cs, ref) <= 1e-13


def test_static_gemm_automatic_split_matches_context_gemm(lib):
    """Deep products with small outputs (Gram matrices, lower triangle only)
    take the split-K path automatically; a second, smaller one follows."""
    import torch
    rng = np.random.default_rng(7)
    ctx = lib.create(8)
    for M, K in ((400, 6000), (96, 2500)):
        Y = _cg(rng, (K, M))
        print(f"static gemm: gram {M}x{M}x{K} automatic", flush=True)
        Gs = lib.zgemm_static(1, 0, _t(Y), _t(Y), _zeros(M, M), flags=16)
        Gc = lib.zgemm(ctx, 1, 0, _t(Y), _t(Y), C=_zeros(M, M), flags=16)
        torch.cuda.synchronize()
        low = np.tril_indices(M)
        ref = (Y.conj().T @ Y)[low]
        gs, gc = _np(Gs)[low], _np(Gc)[low]
        assert _rel(gs, ref) <= 1e-13
        assert _rel(gs, gc) <= 1e-13


def test_static_gemm_rejects_split_beyond_scratch(lib):
    import torch
    M, N, K = 2000, 2000, 64
    A, B, C = _zeros(M, K), _zeros(K, N), _zeros(M, N) + 1
    with pytest.raises(lib.ChfsiError) as e:
        lib.zgemm_static(0, 0, A, B, C, flags=(1 << 8) | (2 << 16))
    assert e.value.status == -1 and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((C == 1).all())
