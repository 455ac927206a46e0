"""Python binding of the gfx950 ChFSI library (``libchfsi.so``).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  PyTorch supplies device memory (complex128 CUDA/HIP tensors)
and the current stream.  The function names mirror the C ABI in
``include/chfsi.h`` without the ``chfsi_`` prefix.

Layout: the C ABI is column-major.  A torch matrix that is not already
column-major is converted (``t.mT.contiguous().mT``) before the call, so a
row-major tensor is never silently read as its (conjugate) transpose.
Results come back as column-major tensors of the logical shape.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchfsi.so")
_lib = None

c_i64, c_i32, c_u32, c_u64, c_dbl, c_vp = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64,
                                           ctypes.c_double, ctypes.c_void_p)

STATUS = {0: "CHFSI_OK", -1: "CHFSI_EINVAL", -2: "CHFSI_ENOTPD", -3: "CHFSI_ENOCONV", -4: "CHFSI_ENAN",
          -5: "CHFSI_ENOMEM", -6: "CHFSI_EHIP"}


class ChfsiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("degree", c_i32), ("max_iter", c_i32), ("lanczos_steps", c_i32), ("precision", c_i32),
                ("seed", c_u64), ("profile", c_i32), ("qr_mode", c_i32),
                ("filter_tile", c_i32), ("filter_splitk", c_i32), ("mixed_switch_digits", c_i32),
                ("reserved", c_i32 * 3)]


class Info(ctypes.Structure):
    _fields_ = [("iterations", c_i32), ("converged", c_i32), ("warm_start", c_i32), ("filter_launches", c_i32),
                ("qr_householder", c_i32), ("reserved_i", c_i32),
                ("filter_flops", c_dbl), ("filter_kernel_seconds", c_dbl),
                ("t_reduce", c_dbl), ("t_lanczos", c_dbl), ("t_filter", c_dbl), ("t_qr", c_dbl), ("t_rr", c_dbl),
                ("t_resid", c_dbl), ("t_total", c_dbl), ("b_upper", c_dbl), ("theta_min", c_dbl), ("h_H", c_dbl),
                ("a0", c_dbl), ("a", c_dbl), ("max_rel_residual", c_dbl),
                ("iterations_fp32", c_i32), ("filter_launches_fp32", c_i32), ("filter_flops_fp32", c_dbl),
                ("filter_kernel_seconds_fp32", c_dbl)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def load():
    """Load libchfsi.so.  Raises if it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1305_5120_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.chfsi_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.chfsi_status_string.restype = ctypes.c_char_p
    L.chfsi_create.argtypes = [ctypes.POINTER(c_vp), c_i64, ctypes.POINTER(Opts), c_vp]
    L.chfsi_release.argtypes = [c_vp]
    L.chfsi_last_error.argtypes = [c_vp]
    L.chfsi_last_error.restype = ctypes.c_char_p
    L.chfsi_reset.argtypes = [c_vp]
    L.chfsi_reduce.argtypes = [c_vp, c_vp, c_i64, c_vp, c_i64]
    L.chfsi_solve.argtypes = [c_vp, c_vp, c_i64, c_vp, c_i64, c_i64, c_i64, c_vp, c_i64, c_i64, c_dbl, c_vp, c_vp, c_i64,
                              ctypes.POINTER(Info)]
    L.chfsi_copy_factors.argtypes = [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64]
    L.chfsi_filter.argtypes = [c_vp, c_vp, c_i64, c_vp, c_i64, c_i64, c_i32, c_dbl, c_dbl, c_dbl]
    L.chfsi_filter_ritz.argtypes = [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_i32, c_dbl, c_dbl,
                                    c_dbl]
    L.chfsi_qr.argtypes = [c_vp, c_vp, c_i64, c_i64]
    L.chfsi_orthonormalize.argtypes = [c_vp, c_vp, c_i64, c_i64, ctypes.POINTER(c_i32)]
    L.chfsi_eigh.argtypes = [c_vp, c_vp, c_i64, c_i64, c_vp, c_vp, c_i64]
    L.chfsi_rayleigh_ritz.argtypes = [c_vp, c_vp, c_i64, c_vp, c_i64, c_i64, c_vp]
    L.chfsi_residuals.argtypes = [c_vp, c_vp, c_i64, c_vp, c_i64, c_vp, c_i64, c_i64, c_vp, c_vp]
    L.chfsi_lanczos.argtypes = [c_vp, c_vp, c_i64, c_i32, c_u64, c_u32, c_vp]
    L.chfsi_random_block.argtypes = [c_vp, c_u64, c_u32, c_i64, c_vp, c_i64, c_i64]
    L.chfsi_philox.argtypes = [c_vp, c_vp, c_vp, c_vp, c_i64]
    L.chfsi_zgemm.argtypes = [c_vp, c_i32, c_i32, c_i64, c_i64, c_i64, c_dbl, c_vp, c_i64, c_vp, c_i64, c_dbl, c_vp,
                              c_i64, c_dbl, c_vp, c_i64, c_vp, c_i64, c_i32]
    L.chfsi_zgemm_static.argtypes = [c_vp, c_i32, c_i32, c_i64, c_i64, c_i64, c_dbl, c_vp, c_i64, c_vp, c_i64, c_dbl,
                                     c_vp, c_i64, c_dbl, c_vp, c_i64, c_vp, c_i64, c_i32]
    for name in ("chfsi_create", "chfsi_reset", "chfsi_reduce", "chfsi_solve", "chfsi_copy_factors", "chfsi_filter",
                 "chfsi_filter_ritz",
                 "chfsi_qr", "chfsi_orthonormalize", "chfsi_eigh", "chfsi_rayleigh_ritz", "chfsi_residuals", "chfsi_lanczos",
                 "chfsi_random_block", "chfsi_philox", "chfsi_zgemm", "chfsi_zgemm_static"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def default_opts(**kw):
    o = Opts()
    load().chfsi_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


# --------------------------------------------------------------------------
# tensor marshalling
# --------------------------------------------------------------------------

def _check_dev(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device (cuda/hip) tensor")
    if t.dtype != torch.complex128:
        raise TypeError(f"{name} must be complex128")
    if t.dim() != 2:
        raise TypeError(f"{name} must be a matrix")


def _check_shape(t, rows, cols, name):
    """Exact logical shape: the C side sees only a pointer and a leading
    dimension, so a larger matrix would be read as its leading block and a
    smaller view would be read past its end."""
    if tuple(t.shape) != (rows, cols):
        raise ValueError(f"{name} must be {rows} x {cols}, got {tuple(t.shape)}")


def colmajor(t):
    """(tensor whose storage is the column-major matrix, leading dimension).
    A tensor with a pending conjugation (``H.conj()``) or negation is
    materialised first, so the pointer holds the values the tensor shows."""
    if t.is_conj():
        t = t.resolve_conj()
    if t.is_neg():
        t = t.resolve_neg()
    rows = t.shape[0]
    if t.stride(0) == 1 and (t.shape[1] <= 1 or t.stride(1) >= max(rows, 1)):
        return t, max(t.stride(1), rows, 1)
    c = t.mT.contiguous().mT
    return c, max(rows, 1)


def empty_colmajor(rows, cols, device):
    import torch
    return torch.empty((cols, rows), dtype=torch.complex128, device=device).mT


def _stream():
    import torch
    return c_vp(torch.cuda.current_stream().cuda_stream)


class Context:
    """Owns one chfsi_ctx (one problem size n, one stream)."""

    def __init__(self, n, opts=None, **kw):
        self.lib = load()
        o = opts if opts is not None else default_opts(**kw)
        h = c_vp()
        st = self.lib.chfsi_create(ctypes.byref(h), int(n), ctypes.byref(o), _stream())
        if st != 0:
            raise ChfsiError(st, "chfsi_create failed")
        self.h = h
        self.n = int(n)
        self.opts = o

    def _raise(self, st):
        if st != 0:
            msg = self.lib.chfsi_last_error(self.h)
            raise ChfsiError(st, msg.decode() if msg else "")

    def release(self):
        if getattr(self, "h", None):
            self.lib.chfsi_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass

    def reset(self):
        self._raise(self.lib.chfsi_reset(self.h))


def create(n, **kw):
    return Context(n, **kw)


def release(ctx):
    ctx.release()


def reset(ctx):
    ctx.reset()


def reduce(ctx, H, S=None):
    _check_dev(H, "H")
    _check_shape(H, ctx.n, ctx.n, "H")
    Hc, ldh = colmajor(H)
    if S is not None:
        _check_dev(S, "S")
        _check_shape(S, ctx.n, ctx.n, "S")
        Sc, lds = colmajor(S)
        sp = Sc.data_ptr()
    else:
        Sc, lds, sp = None, ctx.n, None
    ctx._raise(ctx.lib.chfsi_reduce(ctx.h, Hc.data_ptr(), ldh, sp, lds))


def copy_factors(ctx):
    """Returns (A, L, Linv) of the last reduction as column-major tensors."""
    import torch
    dev = torch.device("cuda")
    A = empty_colmajor(ctx.n, ctx.n, dev)
    L = empty_colmajor(ctx.n, ctx.n, dev)
    Li = empty_colmajor(ctx.n, ctx.n, dev)
    ctx._raise(ctx.lib.chfsi_copy_factors(ctx.h, A.data_ptr(), ctx.n, L.data_ptr(), ctx.n, Li.data_ptr(), ctx.n))
    return A, L, Li


def solve(ctx, H, S, nev, nex, V_warm=None, tol=1e-10, want_vectors=True, raise_on_noconv=True):
    """Algorithm 1 on (H, S).  Returns (evals numpy (nev,), X tensor n x nev
    or None, info dict, status)."""
    _check_dev(H, "H")
    _check_shape(H, ctx.n, ctx.n, "H")
    Hc, ldh = colmajor(H)
    if S is not None:
        _check_dev(S, "S")
        _check_shape(S, ctx.n, ctx.n, "S")
        Sc, lds = colmajor(S)
        sp = Sc.data_ptr()
    else:
        Sc, lds, sp = None, ctx.n, None
    if V_warm is not None:
        _check_dev(V_warm, "V_warm")
        if V_warm.shape[0] != ctx.n or V_warm.shape[1] > nev + nex:
            raise ValueError(f"V_warm must be {ctx.n} x kw with kw <= nev + nex, got {tuple(V_warm.shape)}")
        Vc, ldv = colmajor(V_warm)
        vp, kw = Vc.data_ptr(), V_warm.shape[1]
    else:
        Vc, ldv, vp, kw = None, ctx.n, None, 0
    evals = np.zeros(nev)
    X = empty_colmajor(ctx.n, nev, H.device) if want_vectors else None
    info = Info()
    st = ctx.lib.chfsi_solve(ctx.h, Hc.data_ptr(), ldh, sp, lds, int(nev), int(nex), vp, ldv, int(kw), float(tol),
                             evals.ctypes.data_as(c_vp), X.data_ptr() if X is not None else None, ctx.n,
                             ctypes.byref(info))
    if st != 0 and (raise_on_noconv or st != -3):
        ctx._raise(st)
    return evals, X, info.as_dict(), st


def filter(ctx, A, Y, m, a, b, a0):
    """Y <- p(A) Y (in place on Y, a complex128 device matrix)."""
    _check_dev(A, "A")
    _check_dev(Y, "Y")
    _check_shape(A, ctx.n, ctx.n, "A")
    _check_shape(Y, ctx.n, Y.shape[1], "Y")
    Ac, lda = colmajor(A)
    Yc, ldy = colmajor(Y)
    ctx._raise(ctx.lib.chfsi_filter(ctx.h, Ac.data_ptr(), lda, Yc.data_ptr(), ldy, Y.shape[1], int(m), float(a),
                                    float(b), float(a0)))
    if Yc.data_ptr() != Y.data_ptr():
        Y.copy_(Yc)
    return Y


def filter_ritz(ctx, A, Y, AY, mu, m, a, b, a0):
    """Y <- p(A) Y in place, Y holding Ritz vectors of A with values mu
    (host array) and AY = A Y: the FP32 filter on the Ritz residual."""
    _check_dev(A, "A")
    _check_dev(Y, "Y")
    _check_dev(AY, "AY")
    k = Y.shape[1]
    _check_shape(A, ctx.n, ctx.n, "A")
    _check_shape(Y, ctx.n, k, "Y")
    _check_shape(AY, ctx.n, k, "AY")
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    if mu.shape != (k,):
        raise ValueError(f"mu must hold {k} values, got shape {mu.shape}")
    Ac, lda = colmajor(A)
    Yc, ldy = colmajor(Y)
    AYc, lday = colmajor(AY)
    ctx._raise(ctx.lib.chfsi_filter_ritz(ctx.h, Ac.data_ptr(), lda, Yc.data_ptr(), ldy, AYc.data_ptr(), lday,
                                         mu.ctypes.data_as(c_vp), k, int(m), float(a), float(b), float(a0)))
    if Yc.data_ptr() != Y.data_ptr():
        Y.copy_(Yc)
    return Y


def qr(ctx, Y):
    """Y <- Q (Householder), in place."""
    _check_dev(Y, "Y")
    _check_shape(Y, ctx.n, Y.shape[1], "Y")
    Yc, ldy = colmajor(Y)
    ctx._raise(ctx.lib.chfsi_qr(ctx.h, Yc.data_ptr(), ldy, Y.shape[1]))
    if Yc.data_ptr() != Y.data_ptr():
        Y.copy_(Yc)
    return Y


def orthonormalize(ctx, Y):
    """Y <- orthonormal basis of span(Y), in place (the solver's step).
    Returns True when Householder QR was used."""
    _check_dev(Y, "Y")
    _check_shape(Y, ctx.n, Y.shape[1], "Y")
    Yc, ldy = colmajor(Y)
    used = c_i32(0)
    ctx._raise(ctx.lib.chfsi_orthonormalize(ctx.h, Yc.data_ptr(), ldy, Y.shape[1], ctypes.byref(used)))
    if Yc.data_ptr() != Y.data_ptr():
        Y.copy_(Yc)
    return bool(used.value)


def eigh(ctx, G):
    """(w numpy ascending, Z tensor) of a Hermitian device matrix."""
    _check_dev(G, "G")
    _check_shape(G, G.shape[0], G.shape[0], "G")
    Gc, ldg = colmajor(G)
    k = G.shape[0]
    w = np.zeros(k)
    Z = empty_colmajor(k, k, G.device)
    ctx._raise(ctx.lib.chfsi_eigh(ctx.h, Gc.data_ptr(), ldg, k, w.ctypes.data_as(c_vp), Z.data_ptr(), k))
    return w, Z


def rayleigh_ritz(ctx, A, Y):
    """(mu numpy ascending, Y <- Y Z in place)."""
    _check_dev(A, "A")
    _check_dev(Y, "Y")
    _check_shape(A, ctx.n, ctx.n, "A")
    _check_shape(Y, ctx.n, Y.shape[1], "Y")
    Ac, lda = colmajor(A)
    Yc, ldy = colmajor(Y)
    k = Y.shape[1]
    mu = np.zeros(k)
    ctx._raise(ctx.lib.chfsi_rayleigh_ritz(ctx.h, Ac.data_ptr(), lda, Yc.data_ptr(), ldy, k, mu.ctypes.data_as(c_vp)))
    if Yc.data_ptr() != Y.data_ptr():
        Y.copy_(Yc)
    return mu, Y


def residuals(ctx, A, L, Y, mu):
    _check_dev(A, "A")
    _check_dev(L, "L")
    _check_dev(Y, "Y")
    _check_shape(A, ctx.n, ctx.n, "A")
    _check_shape(L, ctx.n, ctx.n, "L")
    _check_shape(Y, ctx.n, Y.shape[1], "Y")
    if len(mu) != Y.shape[1]:
        raise ValueError("one Ritz value per column of Y")
    Ac, lda = colmajor(A)
    Lc, ldl = colmajor(L)
    Yc, ldy = colmajor(Y)
    k = Y.shape[1]
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    rho = np.zeros(k)
    ctx._raise(ctx.lib.chfsi_residuals(ctx.h, Ac.data_ptr(), lda, Lc.data_ptr(), ldl, Yc.data_ptr(), ldy, k,
                                       mu.ctypes.data_as(c_vp), rho.ctypes.data_as(c_vp)))
    return rho


def lanczos(ctx, A, steps, seed, stream_id):
    _check_dev(A, "A")
    _check_shape(A, ctx.n, ctx.n, "A")
    Ac, lda = colmajor(A)
    out = np.zeros(3)
    ctx._raise(ctx.lib.chfsi_lanczos(ctx.h, Ac.data_ptr(), lda, int(steps), int(seed), int(stream_id),
                                     out.ctypes.data_as(c_vp)))
    return float(out[0]), float(out[1]), float(out[2])


def random_block(ctx, seed, stream_id, k, col0=0):
    import torch
    Y = empty_colmajor(ctx.n, k, torch.device("cuda"))
    ctx._raise(ctx.lib.chfsi_random_block(ctx.h, int(seed), int(stream_id), int(col0), Y.data_ptr(), ctx.n, int(k)))
    return Y


def philox(ctx, ctr, key):
    """Raw Philox4x32-10 blocks for rows of ctr (count x 4) and key (count x 2)."""
    import torch
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    cnt = ctr.shape[0]
    dc = torch.from_numpy(ctr.view(np.int32).copy()).cuda()
    dk = torch.from_numpy(key.view(np.int32).copy()).cuda()
    do = torch.zeros((cnt, 4), dtype=torch.int32, device="cuda")
    ctx._raise(ctx.lib.chfsi_philox(ctx.h, dc.data_ptr(), dk.data_ptr(), do.data_ptr(), cnt))
    return do.cpu().numpy().view(np.uint32)


def zgemm(ctx, opA, opB, A, B, alpha=1.0, beta=0.0, X=None, gamma=0.0, Z=None, C=None, flags=0, M=None, N=None, K=None):
    """C = alpha op(A) op(B) + beta X + gamma Z with the library's kernel."""
    _check_dev(A, "A")
    _check_dev(B, "B")
    Ac, lda = colmajor(A)
    Bc, ldb = colmajor(B)
    M = M if M is not None else (A.shape[0] if opA == 0 else A.shape[1])
    K = K if K is not None else (A.shape[1] if opA == 0 else A.shape[0])
    N = N if N is not None else (B.shape[1] if opB == 0 else B.shape[0])
    # op(A) must hold at least M x K, op(B) K x N, X / Z / C M x N
    ra, ca = (M, K) if opA == 0 else (K, M)
    rb, cb = (K, N) if opB == 0 else (N, K)
    if A.shape[0] < ra or A.shape[1] < ca or B.shape[0] < rb or B.shape[1] < cb:
        raise ValueError("zgemm: A or B smaller than the product's sizes")
    for t, nm in ((X, "X"), (Z, "Z"), (C, "C")):
        if t is not None:
            _check_dev(t, nm)
            if t.shape[0] < M or t.shape[1] < N:
                raise ValueError(f"zgemm: {nm} smaller than M x N")
    if C is None:
        C = empty_colmajor(M, N, A.device)
    Cc, ldc = colmajor(C)
    xp = zp = None
    ldx = ldz = M
    if X is not None:
        Xc, ldx = colmajor(X)
        xp = Xc.data_ptr()
    if Z is not None:
        Zc, ldz = colmajor(Z)
        zp = Zc.data_ptr()
    ctx._raise(ctx.lib.chfsi_zgemm(ctx.h, int(opA), int(opB), int(M), int(N), int(K), float(alpha), Ac.data_ptr(),
                                   lda, Bc.data_ptr(), ldb, float(beta), xp, ldx, float(gamma), zp, ldz,
                                   Cc.data_ptr(), ldc, int(flags)))
    if Cc.data_ptr() != C.data_ptr():
        C.copy_(Cc)
    return C


def zgemm_static(opA, opB, A, B, C, alpha=1.0, beta=0.0, X=None, gamma=0.0, Z=None, flags=0, M=None, N=None,
                 K=None):
    """chfsi_zgemm_static: C = alpha op(A) op(B) + beta X + gamma Z without a
    context and without device allocation in the library (split-K partial
    tiles in its fixed per-GPU scratch), queued on torch's current stream.
    Every tensor must already be a column-major device tensor (the binding
    makes no copies either); C is written in place."""
    import torch
    for t, nm in ((A, "A"), (B, "B"), (C, "C"), (X, "X"), (Z, "Z")):
        if t is None:
            continue
        _check_dev(t, nm)
        if t.stride(0) != 1 or t.stride(1) < max(1, t.shape[0]):
            raise ValueError(f"zgemm_static: {nm} must be column-major (stride (1, ld))")
        if t.is_conj():
            raise ValueError(f"zgemm_static: {nm} has the conjugate bit set")
    M = M if M is not None else (A.shape[0] if opA == 0 else A.shape[1])
    K = K if K is not None else (A.shape[1] if opA == 0 else A.shape[0])
    N = N if N is not None else (B.shape[1] if opB == 0 else B.shape[0])
    ra, ca = (M, K) if opA == 0 else (K, M)
    rb, cb = (K, N) if opB == 0 else (N, K)
    if A.shape[0] < ra or A.shape[1] < ca or B.shape[0] < rb or B.shape[1] < cb:
        raise ValueError("zgemm_static: A or B smaller than the product's sizes")
    for t, nm in ((X, "X"), (Z, "Z"), (C, "C")):
        if t is not None and (t.shape[0] < M or t.shape[1] < N):
            raise ValueError(f"zgemm_static: {nm} smaller than M x N")

    def ld(t):
        return max(1, t.stride(1))

    lib = load()
    stream = torch.cuda.current_stream(C.device).cuda_stream
    st = lib.chfsi_zgemm_static(stream, int(opA), int(opB), int(M), int(N), int(K), float(alpha), A.data_ptr(), ld(A),
                                B.data_ptr(), ld(B), float(beta), X.data_ptr() if X is not None else None,
                                ld(X) if X is not None else int(M), float(gamma),
                                Z.data_ptr() if Z is not None else None, ld(Z) if Z is not None else int(M),
                                C.data_ptr(), ld(C), int(flags))
    if st != 0:
        raise ChfsiError(st, lib.chfsi_last_error(None).decode())
    return C


# --------------------------------------------------------------------------
# serving
# --------------------------------------------------------------------------

class ServerConfig(ctypes.Structure):
    _fields_ = [("workers", c_i32), ("reserved", c_i32), ("hbm_budget_bytes", c_i64), ("opts", Opts)]


class ServerStatistics(ctypes.Structure):
    _fields_ = [("submitted", c_i64), ("completed", c_i64), ("failed", c_i64), ("queued", c_i64), ("running", c_i64),
                ("bytes_in_use", c_i64), ("peak_bytes", c_i64), ("budget_bytes", c_i64),
                ("solves_per_second", c_dbl), ("p50_latency", c_dbl), ("p99_latency", c_dbl), ("mean_latency", c_dbl)]


def _load_server(L):
    if getattr(L, "_server_ready", False):
        return
    L.chfsi_server_create.argtypes = [ctypes.POINTER(c_vp), ctypes.POINTER(ServerConfig)]
    L.chfsi_server_create.restype = ctypes.c_int
    L.chfsi_server_submit.argtypes = [c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_i64, c_i64, c_i64, c_dbl, c_vp, c_vp,
                                      c_i64, ctypes.POINTER(c_i64)]
    L.chfsi_server_submit.restype = ctypes.c_int
    L.chfsi_server_wait.argtypes = [c_vp, c_i64, ctypes.POINTER(Info), ctypes.POINTER(c_dbl)]
    L.chfsi_server_wait.restype = ctypes.c_int
    L.chfsi_server_stats.argtypes = [c_vp, ctypes.POINTER(ServerStatistics)]
    L.chfsi_server_stats.restype = ctypes.c_int
    L.chfsi_server_release_sequence.argtypes = [c_vp, c_i64]
    L.chfsi_server_release_sequence.restype = ctypes.c_int
    L.chfsi_server_last_error.argtypes = [c_vp]
    L.chfsi_server_last_error.restype = ctypes.c_char_p
    L.chfsi_server_destroy.argtypes = [c_vp]
    L._server_ready = True


class Server:
    """Request loop over many sequences (chfsi_server_*).  Inputs stay
    referenced until their ticket is waited for."""

    def __init__(self, workers=4, hbm_budget_bytes=200 << 30, **opts):
        self.lib = load()
        _load_server(self.lib)
        cfg = ServerConfig()
        cfg.workers = workers
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.opts = default_opts(**opts)
        h = c_vp()
        st = self.lib.chfsi_server_create(ctypes.byref(h), ctypes.byref(cfg))
        if st != 0:
            raise ChfsiError(st, "chfsi_server_create failed")
        self.h = h
        self._live = {}

    def submit(self, seq, H, S, nev, nex, tol=1e-10, want_vectors=True):
        """Queue one problem of sequence `seq`.  S = None: the sequence's
        overlap matrix is unchanged since its last request that passed S
        (which must stay valid until this request completes)."""
        import torch
        _check_dev(H, "H")
        n = H.shape[0]
        _check_shape(H, n, n, "H")
        Hc, ldh = colmajor(H)
        if S is not None:
            _check_dev(S, "S")
            _check_shape(S, n, n, "S")
            Sc, lds = colmajor(S)
        else:
            Sc, lds = None, n
        evals = np.zeros(nev)
        X = empty_colmajor(n, nev, H.device) if want_vectors else None
        # the workers run on their own streams: inputs must be complete first
        torch.cuda.current_stream().synchronize()
        t = c_i64()
        st = self.lib.chfsi_server_submit(self.h, int(seq), n, Hc.data_ptr(), ldh,
                                          Sc.data_ptr() if Sc is not None else None, lds, int(nev), int(nex),
                                          float(tol), evals.ctypes.data_as(c_vp),
                                          X.data_ptr() if X is not None else None, n, ctypes.byref(t))
        if st != 0:
            raise ChfsiError(st, "chfsi_server_submit rejected the request")
        self._live[t.value] = (Hc, Sc, evals, X)
        return t.value

    def wait(self, ticket, raise_on_error=True):
        info = Info()
        lat = c_dbl()
        st = self.lib.chfsi_server_wait(self.h, int(ticket), ctypes.byref(info), ctypes.byref(lat))
        Hc, Sc, evals, X = self._live.pop(ticket)
        if st != 0 and raise_on_error:
            msg = self.lib.chfsi_server_last_error(self.h)
            raise ChfsiError(st, msg.decode() if msg else "")
        return evals, X, info.as_dict(), lat.value, st

    def stats(self):
        s = ServerStatistics()
        self.lib.chfsi_server_stats(self.h, ctypes.byref(s))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def release_sequence(self, seq):
        st = self.lib.chfsi_server_release_sequence(self.h, int(seq))
        if st != 0:
            raise ChfsiError(st, "sequence busy")

    def close(self):
        if getattr(self, "h", None):
            self.lib.chfsi_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------
# batching
# --------------------------------------------------------------------------

class BatchReport(ctypes.Structure):
    _fields_ = [("tile_config", c_i32), ("tile_config_fp32", c_i32), ("graph", c_i32), ("outer_iterations", c_i32),
                ("grouped_launches", c_i32), ("converged_members", c_i32), ("filter_flops", c_dbl),
                ("filter_seconds", c_dbl), ("seconds", c_dbl), ("tile_rate", c_dbl * 16)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "tile_rate"}
        d["tile_rate"] = list(self.tile_rate)
        return d


def _load_batch(L):
    if getattr(L, "_batch_ready", False):
        return
    P = ctypes.POINTER
    L.chfsi_batch_create.argtypes = [P(c_vp), c_i32, P(c_i64), P(Opts), c_i32]
    L.chfsi_batch_create.restype = ctypes.c_int
    L.chfsi_batch_solve.argtypes = [c_vp, P(c_vp), P(c_i64), P(c_vp), P(c_i64), P(c_i64), P(c_i64), c_dbl, P(c_vp),
                                    P(c_vp), P(c_i64), P(Info), P(c_i32), P(BatchReport)]
    L.chfsi_batch_solve.restype = ctypes.c_int
    L.chfsi_batch_reset.argtypes = [c_vp]
    L.chfsi_batch_reset.restype = ctypes.c_int
    L.chfsi_batch_last_error.argtypes = [c_vp]
    L.chfsi_batch_last_error.restype = ctypes.c_char_p
    L.chfsi_batch_release.argtypes = [c_vp]
    L._batch_ready = True


class Batch:
    """Lockstep solver for a fixed set of independent problems whose filters
    share grouped launches (chfsi_batch_*).  Member i solves problems of size
    sizes[i] and keeps its warm state between calls."""

    def __init__(self, sizes, use_graph=True, **opts):
        self.lib = load()
        _load_batch(self.lib)
        self.sizes = [int(n) for n in sizes]
        arr = (c_i64 * len(self.sizes))(*self.sizes)
        o = default_opts(**opts)
        h = c_vp()
        st = self.lib.chfsi_batch_create(ctypes.byref(h), len(self.sizes), arr, ctypes.byref(o), 1 if use_graph else 0)
        if st != 0:
            raise ChfsiError(st, "chfsi_batch_create failed")
        self.h = h

    def solve(self, H, S, nev, nex, tol=1e-10, want_vectors=True, raise_on_error=True):
        """H, S: lists of device matrices (S entries may be None); nev, nex:
        lists of ints.  Returns (evals list, X list, infos, statuses, report)."""
        import torch
        G = len(self.sizes)
        if not (len(H) == len(S) == len(nev) == len(nex) == G):
            raise ValueError("one H, S, nev, nex per member")
        keep = []
        hp, lh, sp, ls, xp, lx, ev = [], [], [], [], [], [], []
        evals, Xs = [], []
        for i in range(G):
            n = self.sizes[i]
            _check_dev(H[i], f"H[{i}]")
            if H[i].shape != (n, n):
                raise ValueError(f"H[{i}] must be {n} x {n}")
            Hc, ldh = colmajor(H[i])
            keep.append(Hc)
            hp.append(Hc.data_ptr())
            lh.append(ldh)
            if S[i] is not None:
                _check_dev(S[i], f"S[{i}]")
                _check_shape(S[i], n, n, f"S[{i}]")
                Sc, lds = colmajor(S[i])
                keep.append(Sc)
                sp.append(Sc.data_ptr())
                ls.append(lds)
            else:
                sp.append(None)
                ls.append(n)
            e = np.zeros(int(nev[i]))
            evals.append(e)
            ev.append(e.ctypes.data)
            X = empty_colmajor(n, int(nev[i]), H[i].device) if want_vectors else None
            Xs.append(X)
            xp.append(X.data_ptr() if X is not None else None)
            lx.append(n)
        torch.cuda.current_stream().synchronize()
        infos = (Info * G)()
        stats = (c_i32 * G)()
        rep = BatchReport()
        st = self.lib.chfsi_batch_solve(self.h, (c_vp * G)(*hp), (c_i64 * G)(*lh), (c_vp * G)(*sp), (c_i64 * G)(*ls),
                                        (c_i64 * G)(*[int(v) for v in nev]), (c_i64 * G)(*[int(v) for v in nex]),
                                        float(tol), (c_vp * G)(*ev), (c_vp * G)(*xp), (c_i64 * G)(*lx), infos, stats,
                                        ctypes.byref(rep))
        if st != 0 and raise_on_error:
            msg = self.lib.chfsi_batch_last_error(self.h)
            raise ChfsiError(st, msg.decode() if msg else "")
        return evals, Xs, [infos[i].as_dict() for i in range(G)], list(stats), rep.as_dict()

    def reset(self):
        self.lib.chfsi_batch_reset(self.h)

    def close(self):
        if getattr(self, "h", None):
            self.lib.chfsi_batch_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
