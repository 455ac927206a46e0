"""CPU oracle for the Chebyshev-filtered subspace iteration (arXiv 1305.5120).

TEST INFRASTRUCTURE ONLY: the parity tests, the smoke check and the
CPU-baseline leg of the benchmark call it; the product path (the HIP library
and its binding) never imports it.  It shares no code with the GPU path.

Every function takes and returns numpy arrays; matrices are complex128 and
are handed to the C code in column-major (Fortran) order.  Each wrapper
names the part of the paper its C routine follows.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

c_i64 = ctypes.c_int64
c_dbl = ctypes.c_double
c_vp = ctypes.c_void_p


class OrcOpts(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("lanczos_steps", ctypes.c_int32), ("have_bounds", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class OrcInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("status", ctypes.c_int32), ("bad_column", ctypes.c_int32),
                ("b_upper", c_dbl), ("theta_min", c_dbl), ("h_H", c_dbl),
                ("a0", c_dbl), ("a", c_dbl), ("filter_flops", c_dbl),
                ("max_rel_residual", c_dbl)]


def lib():
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [c_vp, c_vp, c_vp]
        L.orc_gauss_block.argtypes = [ctypes.c_uint64, ctypes.c_uint32, c_i64, c_i64, c_i64, c_vp, c_i64]
        L.orc_cholesky.argtypes = [c_i64, c_vp, c_i64, c_vp, c_i64]
        L.orc_cholesky.restype = c_i64
        L.orc_reduce.argtypes = [c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64]
        L.orc_backtransform.argtypes = [c_i64, c_i64, c_vp, c_i64, c_vp, c_i64]
        L.orc_lh_times.argtypes = [c_i64, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64]
        L.orc_jacobi_eigh.argtypes = [c_i64, c_vp, c_i64, c_vp, c_vp, c_i64]
        L.orc_jacobi_eigh.restype = ctypes.c_int
        L.orc_householder_qr.argtypes = [c_i64, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64]
        L.orc_lanczos.argtypes = [c_i64, c_vp, c_i64, c_i64, c_vp, c_vp]
        L.orc_filter.argtypes = [c_i64, c_vp, c_i64, c_vp, c_i64, c_i64, ctypes.c_int32, c_dbl, c_dbl, c_dbl]
        L.orc_rayleigh_ritz.argtypes = [c_i64, c_vp, c_i64, c_vp, c_i64, c_i64, c_vp]
        L.orc_residuals.argtypes = [c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_i64, c_vp, c_vp]
        L.orc_solve.argtypes = [c_i64, c_vp, c_i64, c_vp, c_i64, c_i64, c_i64, c_vp, c_i64, c_i64, c_vp,
                                c_dbl, ctypes.POINTER(OrcOpts), c_vp, c_vp, c_i64, c_vp, ctypes.POINTER(OrcInfo)]
        L.orc_solve.restype = ctypes.c_int32
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _f(a):
    """complex128 Fortran-ordered copy (the C code's column-major layout)."""
    return np.array(a, dtype=np.complex128, order="F", copy=True)


def _p(a):
    return a.ctypes.data_as(c_vp)


def set_threads(n):
    """Threads of the oracle's OpenMP loops (n < 1: unchanged); returns the
    previous count."""
    return int(lib().orc_set_threads(int(n)))


def philox4x32_10(ctr, key):
    """Raw Philox4x32-10 block (four uint32) for counter ``ctr`` and ``key``."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def gauss_block(seed, stream, n, k, col0=0):
    """n x k complex Gaussian block of the counter-based stream (column j of
    the result is column col0 + j of the stream)."""
    Y = np.zeros((n, k), dtype=np.complex128, order="F")
    lib().orc_gauss_block(seed, stream, n, k, col0, _p(Y), n)
    return Y


def cholesky(S):
    """S = L L^H (reduction to standard form).  Returns (L, bad) where bad is 0
    or the 1-based column whose pivot was not positive."""
    S = _f(S)
    n = S.shape[0]
    L = np.zeros((n, n), dtype=np.complex128, order="F")
    bad = lib().orc_cholesky(n, _p(S), n, _p(L), n)
    return L, int(bad)


def reduce(H, L):
    """A = L^{-1} H L^{-H}, Hermitian part (reduction to standard form)."""
    H = _f(H)
    L = _f(L)
    n = H.shape[0]
    A = np.zeros((n, n), dtype=np.complex128, order="F")
    lib().orc_reduce(n, _p(H), n, _p(L), n, _p(A), n)
    return A


def backtransform(L, Y):
    """X = L^{-H} Y."""
    L = _f(L)
    X = _f(Y)
    n, k = X.shape
    lib().orc_backtransform(n, k, _p(L), n, _p(X), n)
    return X


def lh_times(L, V):
    """Y = L^H V (warm-start vectors mapped into the standard form)."""
    L = _f(L)
    V = _f(V)
    n, k = V.shape
    Y = np.zeros((n, k), dtype=np.complex128, order="F")
    lib().orc_lh_times(n, k, _p(L), n, _p(V), n, _p(Y), n)
    return Y


def jacobi_eigh(G):
    """Cyclic Jacobi eigensolver: returns (w ascending, Z, sweeps)."""
    G = _f(G)
    k = G.shape[0]
    w = np.zeros(k)
    Z = np.zeros((k, k), dtype=np.complex128, order="F")
    sweeps = lib().orc_jacobi_eigh(k, _p(G), k, _p(w), _p(Z), k)
    return w, Z, int(sweeps)


def householder_qr(Y):
    """Householder QR: returns (Q n x k, R k x k upper, real diagonal)."""
    Y = _f(Y)
    n, k = Y.shape
    Q = np.zeros((n, k), dtype=np.complex128, order="F")
    R = np.zeros((k, k), dtype=np.complex128, order="F")
    lib().orc_householder_qr(n, k, _p(Y), n, _p(Q), n, _p(R), k)
    return Q, R


def lanczos(A, steps, v0):
    """Lanczos with full re-orthogonalization.  Returns
    (theta_min, theta_max, upper_bound)."""
    A = _f(A)
    v0 = np.array(v0, dtype=np.complex128).reshape(-1).copy()
    n = A.shape[0]
    out = np.zeros(3)
    lib().orc_lanczos(n, _p(A), n, steps, _p(v0), _p(out))
    return float(out[0]), float(out[1]), float(out[2])


def chebyshev_filter(A, Y, m, a, b, a0):
    """Scaled Chebyshev filter of degree m: returns p(A) Y with
    p(t) = C_m((t-c)/e) / C_m((a0-c)/e), c = (a+b)/2, e = (b-a)/2."""
    A = _f(A)
    Y = _f(Y)
    n, k = Y.shape
    lib().orc_filter(n, _p(A), n, _p(Y), n, k, m, a, b, a0)
    return Y


def rayleigh_ritz(A, Y):
    """Rayleigh-Ritz on the orthonormal block Y: returns (mu ascending, Y Z)."""
    A = _f(A)
    Y = _f(Y)
    n, k = Y.shape
    mu = np.zeros(k)
    lib().orc_rayleigh_ritz(n, _p(A), n, _p(Y), n, k, _p(mu))
    return mu, Y


def residuals(A, L, Y, mu):
    """rho_j = ||L (A y_j - mu_j y_j)||_2 = ||H x_j - mu_j S x_j||_2."""
    A = _f(A)
    L = _f(L)
    Y = _f(Y)
    n, k = Y.shape
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    rho = np.zeros(k)
    lib().orc_residuals(n, _p(A), n, _p(L), n, _p(Y), n, k, _p(mu), _p(rho))
    return rho


def solve(H, S, nev, nex, tol=1e-10, degree=10, max_iter=1000, lanczos_steps=10, seed=0,
          V_warm=None, bounds=None):
    """Algorithm 1 (ChFSI with locking) on the pencil (H, S).

    Returns a dict with ``evals`` (nev), ``X`` (n x nev generalized
    eigenvectors), ``Y`` (n x (nev+nex) final standard-form block, the warm
    state), ``info`` (iteration counts, bounds, status)."""
    H = _f(H)
    S = _f(S)
    n = H.shape[0]
    k = nev + nex
    opts = OrcOpts(degree, max_iter, lanczos_steps, 1 if bounds is not None else 0, seed)
    info = OrcInfo()
    evals = np.zeros(nev)
    X = np.zeros((n, nev), dtype=np.complex128, order="F")
    Y = np.zeros((n, k), dtype=np.complex128, order="F")
    if V_warm is not None:
        Vw = _f(V_warm)
        kw = Vw.shape[1]
        vp = _p(Vw)
    else:
        Vw = None
        kw = 0
        vp = None
    bnd = np.array(bounds if bounds is not None else [0.0, 0.0], dtype=np.float64)
    st = lib().orc_solve(n, _p(H), n, _p(S), n, nev, nex, vp, n, kw, _p(bnd), tol, ctypes.byref(opts),
                         _p(evals), _p(X), n, _p(Y), ctypes.byref(info))
    d = {f: getattr(info, f) for f, _ in OrcInfo._fields_}
    d["status"] = int(st)
    return {"evals": evals, "X": X, "Y": Y, "info": d}
