"""Python binding of libmfeast.so (Hermitian FEAST contour-integration eigensolver, MI355X).

Argument marshalling only: every numerical step runs in the HIP kernels of the
library.  PyTorch provides device memory and the stream.  The functions named like
the C entry points (``mfeast_*``) map one to one onto ``include/mfeast.h``;
``feast`` is a convenience wrapper that allocates the outputs.

If the compiled library is missing the import still succeeds (so CPU-only tools can
read the module), but every call raises: there is no fallback implementation.
"""

import ctypes
import sys
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfeast.so")

_lib = None
_lib_error = None

EXPORTED = (
    "mfeast_create", "mfeast_destroy", "mfeast_set_stream", "mfeast_init", "mfeast_init_ifeast",
    "mfeast_init_stochastic", "mfeast_contour", "mfeast_zolotarev", "mfeast_dsygv", "mfeast_dsygv_noalloc",
    "mfeast_zhegv", "mfeast_dcsrgv", "mfeast_dsy_adjoint", "mfeast_dsygv_batched", "mfeast_get_timing",
    "mfeast_get_profile", "mfeast_set_profiling", "mfeast_init_general", "mfeast_gcontour", "mfeast_zgegv",
    "mfeast_init_polynomial", "mfeast_zgepev",
)


def _load():
    global _lib, _lib_error
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        _lib_error = "libmfeast.so not built (run __graft_entry__.build())"
        raise RuntimeError(_lib_error)
    lib = ctypes.CDLL(LIB_PATH)
    c_int, c_i32p, c_dp, c_vp = ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p, ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.mfeast_create.argtypes = [ctypes.POINTER(c_vp), c_int, c_vp]
    lib.mfeast_create.restype = c_int
    lib.mfeast_destroy.argtypes = [c_vp]
    lib.mfeast_destroy.restype = c_int
    lib.mfeast_set_stream.argtypes = [c_vp, c_vp]
    lib.mfeast_set_stream.restype = c_int
    lib.mfeast_init.argtypes = [c_i32p]
    lib.mfeast_init.restype = None
    lib.mfeast_init_ifeast.argtypes = [c_i32p]
    lib.mfeast_init_ifeast.restype = None
    lib.mfeast_init_stochastic.argtypes = [c_i32p]
    lib.mfeast_init_stochastic.restype = None
    lib.mfeast_contour.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, c_dp, c_dp]
    lib.mfeast_contour.restype = c_int
    lib.mfeast_zolotarev.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, c_dp, c_dp,
                                     ctypes.POINTER(ctypes.c_double)]
    lib.mfeast_zolotarev.restype = c_int
    lib.mfeast_init_general.argtypes = [c_i32p]
    lib.mfeast_init_general.restype = None
    lib.mfeast_gcontour.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, c_dp, c_dp]
    lib.mfeast_gcontour.restype = c_int
    lib.mfeast_zgegv.argtypes = [c_vp, i64, c_dp, i64, c_dp, i64, c_i32p, ctypes.POINTER(ctypes.c_double), c_i32p,
                                 c_dp, ctypes.c_double, c_i32p, c_dp, c_dp, i64, c_i32p, c_dp, c_dp, c_dp]
    lib.mfeast_zgegv.restype = c_int
    lib.mfeast_init_polynomial.argtypes = [c_i32p]
    lib.mfeast_init_polynomial.restype = None
    lib.mfeast_zgepev.argtypes = [c_vp, ctypes.c_int32, i64, c_dp, i64, c_i32p, ctypes.POINTER(ctypes.c_double),
                                  c_i32p, c_dp, ctypes.c_double, c_i32p, c_dp, c_dp, i64, c_i32p, c_dp, c_dp, c_dp]
    lib.mfeast_zgepev.restype = c_int
    dense = [c_vp, ctypes.c_char, i64, c_dp, i64, c_dp, i64, c_i32p, ctypes.c_double, ctypes.c_double,
             c_i32p, c_dp, c_dp, i64, c_i32p, c_dp, ctypes.POINTER(ctypes.c_double), c_i32p, c_dp, c_dp]
    for name in ("mfeast_dsygv", "mfeast_zhegv", "mfeast_dsygv_noalloc"):
        fn = getattr(lib, name)
        fn.argtypes = dense
        fn.restype = c_int
    lib.mfeast_dcsrgv.argtypes = [c_vp, ctypes.c_char, i64, c_dp, c_vp, c_vp, ctypes.c_int32, c_dp, c_vp, c_vp,
                                  c_i32p, ctypes.c_double, ctypes.c_double, c_i32p, c_dp, c_dp, i64, c_i32p, c_dp,
                                  ctypes.POINTER(ctypes.c_double), c_i32p, c_dp, c_dp]
    lib.mfeast_dcsrgv.restype = c_int
    lib.mfeast_dsy_adjoint.argtypes = [c_vp, i64, c_dp, i64, ctypes.c_int32, c_dp, c_dp, i64, c_dp, c_dp, i64,
                                       ctypes.c_int32, c_dp, i64, c_dp]
    lib.mfeast_dsy_adjoint.restype = c_int
    pp = ctypes.POINTER(ctypes.c_void_p)
    i64p = ctypes.POINTER(ctypes.c_int64)
    dpp = ctypes.POINTER(ctypes.c_double)
    lib.mfeast_dsygv_batched.argtypes = [c_vp, ctypes.c_int32, i64p, pp, i64p, pp, i64p, c_i32p, dpp, dpp, c_i32p,
                                         pp, pp, i64p, c_i32p, pp, dpp, c_i32p, c_i32p]
    lib.mfeast_dsygv_batched.restype = c_int
    lib.mfeast_get_timing.argtypes = [c_vp, ctypes.POINTER(ctypes.c_double)]
    lib.mfeast_get_timing.restype = c_int
    lib.mfeast_set_profiling.argtypes = [c_vp, ctypes.c_int32]
    lib.mfeast_set_profiling.restype = c_int
    lib.mfeast_get_profile.argtypes = [c_vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int32]
    lib.mfeast_get_profile.restype = c_int
    _lib = lib
    return lib


def library():
    """The loaded ctypes library (raises if it is not built)."""
    return _load()


# ----------------------------------------------------------------------------- helpers

def _ptr(t):
    """Device (or host) address of a tensor / ndarray, or None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _fpm_array(fpm):
    arr = np.ascontiguousarray(np.asarray(fpm, dtype=np.int32))
    if arr.size != 64:
        raise ValueError("fpm must have 64 entries")
    return arr


def mfeast_init():
    """Default fpm[64] (feastinit) as an int32 numpy array."""
    fpm = np.zeros(64, dtype=np.int32)
    _load().mfeast_init(fpm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return fpm


def mfeast_init_ifeast():
    """IFEAST defaults of fpm[64] as an int32 numpy array."""
    fpm = np.zeros(64, dtype=np.int32)
    _load().mfeast_init_ifeast(fpm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return fpm


def mfeast_init_stochastic():
    """fpm[64] defaults of the stochastic eigenvalue-count mode (fpm(14)=2)."""
    fpm = np.zeros(64, dtype=np.int32)
    _load().mfeast_init_stochastic(fpm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return fpm


def mfeast_contour(emin, emax, ne, rule=0, ratio_pct=30):
    """(info, z, w): half-contour nodes and weights as complex128 arrays."""
    zb = np.zeros(2 * max(int(ne), 1), dtype=np.float64)
    wb = np.zeros_like(zb)
    info = _load().mfeast_contour(float(emin), float(emax), int(ne), int(rule), int(ratio_pct),
                                  zb.ctypes.data, wb.ctypes.data)
    return info, zb.view(np.complex128)[:ne].copy(), wb.view(np.complex128)[:ne].copy()


def mfeast_zolotarev(emin, emax, ne, band_pct=90):
    """(info, z, w, c_inf): Zolotarev nodes, half-contour weights and constant term."""
    zb = np.zeros(2 * max(int(ne), 1), dtype=np.float64)
    wb = np.zeros_like(zb)
    c = ctypes.c_double(0.0)
    info = _load().mfeast_zolotarev(float(emin), float(emax), int(ne), int(band_pct), zb.ctypes.data,
                                    wb.ctypes.data, ctypes.byref(c))
    return info, zb.view(np.complex128)[:ne].copy(), wb.view(np.complex128)[:ne].copy(), c.value


def mfeast_init_general():
    """fpm defaults of the non-Hermitian driver (two-sided, trapezoidal, circle)."""
    fpm = np.zeros(64, dtype=np.int32)
    _load().mfeast_init_general(fpm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return fpm


def mfeast_init_polynomial():
    """fpm defaults of the polynomial driver (right eigenvectors, trapezoidal, circle)."""
    fpm = np.zeros(64, dtype=np.int32)
    _load().mfeast_init_polynomial(fpm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return fpm


def mfeast_gcontour(emid, r, ne, rule=1, ratio_pct=100, angle_deg=0):
    """(info, z, w): full-contour nodes and weights as complex128 arrays."""
    zb = np.zeros(2 * max(int(ne), 1), dtype=np.float64)
    wb = np.zeros_like(zb)
    emid = complex(emid)
    info = _load().mfeast_gcontour(emid.real, emid.imag, float(r), int(ne), int(rule), int(ratio_pct), int(angle_deg),
                                   zb.ctypes.data, wb.ctypes.data)
    return info, zb.view(np.complex128)[:ne].copy(), wb.view(np.complex128)[:ne].copy()


class Handle:
    """Owns an mfeast handle bound to a device and a HIP stream (torch's current by default)."""

    def __init__(self, device=0, stream=None):
        import torch
        lib = _load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        h = ctypes.c_void_p()
        info = lib.mfeast_create(ctypes.byref(h), int(device), ctypes.c_void_p(raw))
        if info != 0:
            raise RuntimeError("mfeast_create failed with info %d" % info)
        self.ptr = h
        self.device = device

    def close(self):
        if self.ptr is not None and self.ptr.value:
            _load().mfeast_destroy(self.ptr)
        self.ptr = None

    def __del__(self):
        # no HIP call while the interpreter shuts down: the runtime (and a profiler's tool
        # library) may already be finalized; the process exit releases the device memory.
        # A closed handle has nothing to release (and at shutdown the module globals,
        # sys included, may already be gone).
        if getattr(self, "ptr", None) is None or sys is None or sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def timing(self):
        out = (ctypes.c_double * 8)()
        _load().mfeast_get_timing(self.ptr, out)
        return list(out)

    PROFILE_CLASSES = ("lu_trailing_gemm", "lu_panel", "contour_solve", "rr_gemm", "reduced_eig", "other",
                       "bicgstab_spmv", "bicgstab_vector", "orth", "lu_rows", "resid", "batched_factor")

    def set_profiling(self, on=True):
        """Per-class device timing of every later call on this handle (mfeast_set_profiling)."""
        info = _load().mfeast_set_profiling(self.ptr, 1 if on else 0)
        if info != 0:
            raise RuntimeError("mfeast_set_profiling failed with info %d" % info)

    def profile(self):
        """Per-class device timing of the last call made with fpm[51] = 1."""
        k = 4 * len(self.PROFILE_CLASSES)
        out = (ctypes.c_double * k)()
        _load().mfeast_get_profile(self.ptr, out, k)
        return {name: {"launches": out[4 * i], "ms": out[4 * i + 1], "flops": out[4 * i + 2],
                       "bytes": out[4 * i + 3]} for i, name in enumerate(self.PROFILE_CLASSES)}


def _dense_call(name, h, uplo, n, A, lda, B, ldb, fpm, emin, emax, m0, E, X, ldx, res, zne=None, wne=None):
    lib = _load()
    fpm_a = _fpm_array(fpm)
    m0_c = ctypes.c_int32(int(m0))
    M_c = ctypes.c_int32(0)
    eps_c = ctypes.c_double(0.0)
    loop_c = ctypes.c_int32(0)
    zb = wb = None
    if zne is not None:
        zb = np.ascontiguousarray(np.asarray(zne, dtype=np.complex128)).view(np.float64)
        wb = np.ascontiguousarray(np.asarray(wne, dtype=np.complex128)).view(np.float64)
    hp = h.ptr if isinstance(h, Handle) else h
    info = getattr(lib, name)(
        hp, uplo.encode() if isinstance(uplo, str) else uplo, int(n), _ptr(A), int(lda), _ptr(B), int(ldb),
        fpm_a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), float(emin), float(emax), ctypes.byref(m0_c),
        _ptr(E), _ptr(X), int(ldx), ctypes.byref(M_c), _ptr(res), ctypes.byref(eps_c), ctypes.byref(loop_c),
        None if zb is None else zb.ctypes.data, None if wb is None else wb.ctypes.data)
    if isinstance(fpm, np.ndarray) and fpm.dtype == np.int32 and fpm.size == 64:
        fpm[:] = fpm_a
    return {"info": int(info), "m0": int(m0_c.value), "M": int(M_c.value), "epsout": float(eps_c.value),
            "loop": int(loop_c.value)}


def mfeast_dsygv(h, uplo, n, A, lda, B, ldb, fpm, emin, emax, m0, E, X, ldx, res, zne=None, wne=None):
    """C mfeast_dsygv; A, B, E, X, res are device tensors (column-major A, B, X)."""
    return _dense_call("mfeast_dsygv", h, uplo, n, A, lda, B, ldb, fpm, emin, emax, m0, E, X, ldx, res, zne, wne)


def mfeast_dsygv_noalloc(h, uplo, n, A, lda, B, ldb, fpm, emin, emax, m0, E, X, ldx, res, zne=None, wne=None):
    """C mfeast_dsygv_noalloc: mfeast_dsygv with its workspace in the library's static
    device array (no device allocation); -901 when the problem does not fit it."""
    return _dense_call("mfeast_dsygv_noalloc", h, uplo, n, A, lda, B, ldb, fpm, emin, emax, m0, E, X, ldx, res,
                       zne, wne)


def mfeast_zhegv(h, uplo, n, A, lda, B, ldb, fpm, emin, emax, m0, E, X, ldx, res, zne=None, wne=None):
    """C mfeast_zhegv; complex128 device tensors (interleaved re, im)."""
    return _dense_call("mfeast_zhegv", h, uplo, n, A, lda, B, ldb, fpm, emin, emax, m0, E, X, ldx, res, zne, wne)


def mfeast_dcsrgv(h, uplo, n, a, ia, ja, index_base, b, ib, jb, fpm, emin, emax, m0, E, X, ldx, res,
                  zne=None, wne=None):
    """C mfeast_dcsrgv; a, ia, ja (and b, ib, jb or None) are device tensors (float64, int32)."""
    lib = _load()
    fpm_a = _fpm_array(fpm)
    m0_c = ctypes.c_int32(int(m0))
    M_c = ctypes.c_int32(0)
    eps_c = ctypes.c_double(0.0)
    loop_c = ctypes.c_int32(0)
    zb = wb = None
    if zne is not None:
        zb = np.ascontiguousarray(np.asarray(zne, dtype=np.complex128)).view(np.float64)
        wb = np.ascontiguousarray(np.asarray(wne, dtype=np.complex128)).view(np.float64)
    hp = h.ptr if isinstance(h, Handle) else h
    info = lib.mfeast_dcsrgv(
        hp, uplo.encode() if isinstance(uplo, str) else uplo, int(n), _ptr(a), _ptr(ia), _ptr(ja),
        int(index_base), _ptr(b), _ptr(ib), _ptr(jb), fpm_a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        float(emin), float(emax), ctypes.byref(m0_c), _ptr(E), _ptr(X), int(ldx), ctypes.byref(M_c), _ptr(res),
        ctypes.byref(eps_c), ctypes.byref(loop_c), None if zb is None else zb.ctypes.data,
        None if wb is None else wb.ctypes.data)
    if isinstance(fpm, np.ndarray) and fpm.dtype == np.int32 and fpm.size == 64:
        fpm[:] = fpm_a
    return {"info": int(info), "m0": int(m0_c.value), "M": int(M_c.value), "epsout": float(eps_c.value),
            "loop": int(loop_c.value), "fpm60": int(fpm_a[59])}


def mfeast_dsy_adjoint(h, n, A, lda, M, E, X, ldx, gE, gX, ldgx, precision, gA, ldga, gdiag):
    """C mfeast_dsy_adjoint; returns info."""
    hp = h.ptr if isinstance(h, Handle) else h
    return int(_load().mfeast_dsy_adjoint(hp, int(n), _ptr(A), int(lda), int(M), _ptr(E), _ptr(X), int(ldx),
                                          _ptr(gE), _ptr(gX), int(ldgx), int(precision), _ptr(gA), int(ldga),
                                          _ptr(gdiag)))


def colmajor(t):
    """(tensor, leading dimension) with element (i, j) at i + j*ld; copies only if needed."""
    if t.dim() != 2:
        raise ValueError("expected a matrix")
    if t.stride(0) == 1 and t.stride(1) >= t.shape[0]:
        return t, t.stride(1)
    c = t.mT.contiguous().mT
    return c, c.stride(1)


def feast(A, B, emin, emax, m0, fpm=None, X0=None, uplo="F", handle=None, zne=None, wne=None):
    """Eigenpairs of A x = lambda B x with lambda in [emin, emax] (B None means identity).

    A, B: torch tensors on the GPU (float64 or complex128).  Returns a dict with E, X
    (n x M0 column-major tensor), res, M, m0, loop, epsout, info.  fpm defaults to
    mfeast_init(); X0 (with fpm[4] = 1) is the starting subspace.
    """
    import torch
    n = A.shape[0]
    cplx = A.is_complex() or (B is not None and B.is_complex())
    dt = torch.complex128 if cplx else torch.float64
    dev = A.device
    fpm = mfeast_init() if fpm is None else _fpm_array(fpm).copy()
    A_, lda = colmajor(A.to(dt))
    B_, ldb = (None, n) if B is None else colmajor(B.to(dt))
    X = torch.zeros((m0, n), dtype=dt, device=dev).mT
    if X0 is not None:
        X.copy_(X0.to(dt))
        fpm[4] = 1
    E = torch.zeros(m0, dtype=torch.float64, device=dev)
    res = torch.zeros(m0, dtype=torch.float64, device=dev)
    own = handle is None
    h = Handle(dev.index or 0) if own else handle
    try:
        fn = mfeast_zhegv if cplx else mfeast_dsygv
        out = fn(h, uplo, n, A_, lda, B_, ldb, fpm, emin, emax, m0, E, X, n, res, zne, wne)
        out["timing"] = h.timing()
        if fpm[51] == 1:
            out["profile"] = h.profile()
    finally:
        if own:
            h.close()
    m = out["m0"]
    out.update(E=E[:m], X=X[:, :m], res=res[:m], fpm=fpm)
    return out


def feast_csr(csr, emin, emax, m0, fpm=None, B=None, X0=None, uplo="F", index_base=0, handle=None,
              zne=None, wne=None, device=0):
    """IFEAST on a real symmetric CSR matrix: csr = (values, row pointers, column indices)
    as numpy arrays or device tensors (float64, int32, int32); B likewise or None.

    Returns the dict of mfeast_dcsrgv plus E, X (n x M0 column-major tensor), res, fpm.
    fpm defaults to mfeast_init_ifeast().
    """
    import torch
    dev = torch.device("cuda", device)

    def dev_arr(x, dt):
        return x.to(dev, dt) if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x), dtype=dt, device=dev)

    a, ia, ja = dev_arr(csr[0], torch.float64), dev_arr(csr[1], torch.int32), dev_arr(csr[2], torch.int32)
    n = ia.numel() - 1
    b = ib = jb = None
    if B is not None:
        b, ib, jb = dev_arr(B[0], torch.float64), dev_arr(B[1], torch.int32), dev_arr(B[2], torch.int32)
    fpm = mfeast_init_ifeast() if fpm is None else _fpm_array(fpm).copy()
    X = torch.zeros((m0, n), dtype=torch.float64, device=dev).mT
    if X0 is not None:
        X.copy_(X0.to(torch.float64))
        fpm[4] = 1
    E = torch.zeros(m0, dtype=torch.float64, device=dev)
    res = torch.zeros(m0, dtype=torch.float64, device=dev)
    own = handle is None
    h = Handle(device) if own else handle
    try:
        out = mfeast_dcsrgv(h, uplo, n, a, ia, ja, index_base, b, ib, jb, fpm, emin, emax, m0, E, X, n, res,
                            zne, wne)
        out["timing"] = h.timing()
        if fpm[51] == 1:
            out["profile"] = h.profile()
    finally:
        if own:
            h.close()
    m = out["m0"]
    out.update(E=E[:m], X=X[:, :m], res=res[:m], fpm=fpm)
    return out


def _feast_eigh_class():
    import torch

    class FeastEigh(torch.autograd.Function):
        """Eigenpairs of a real symmetric A inside [emin, emax] (mfeast_dsygv) with a
        backward pass by mfeast_dsy_adjoint (dL/dA for losses invariant under rotations
        inside the span of the returned eigenvectors)."""

        @staticmethod
        def forward(ctx, A, emin, emax, m0, fpm, precision, handle):
            out = feast(A, None, emin, emax, m0, fpm=fpm, handle=handle)
            if out["info"] != 0:
                raise RuntimeError("mfeast_dsygv returned info %d" % out["info"])
            M = out["M"]
            E = out["E"][:M].clone()
            X = out["X"][:, :M].clone()
            ctx.save_for_backward(A, E, X)
            ctx.precision = precision
            ctx.handle = handle
            return E, X

        @staticmethod
        def backward(ctx, gE, gX):
            A, E, X = ctx.saved_tensors
            n, M = X.shape
            Ac, lda = colmajor(A.to(torch.float64))
            Xc, ldx = colmajor(X)
            gEc = None if gE is None else gE.to(torch.float64).contiguous()
            gXc, ldgx = (None, n) if gX is None else colmajor(gX.to(torch.float64))
            gA = torch.empty((n, n), dtype=torch.float64, device=A.device)
            own = ctx.handle is None
            h = Handle(A.device.index or 0) if own else ctx.handle
            try:
                info = mfeast_dsy_adjoint(h, n, Ac, lda, M, E, Xc, ldx, gEc, gXc, ldgx, ctx.precision, gA, n, None)
            finally:
                if own:
                    h.close()
            if info != 0:
                raise RuntimeError("mfeast_dsy_adjoint returned info %d" % info)
            return gA, None, None, None, None, None, None

    return FeastEigh


_FEAST_EIGH = None


def feast_eigh(A, emin, emax, m0, fpm=None, precision=1, handle=None):
    """(E, X) of the eigenpairs of real symmetric A in [emin, emax], differentiable:
    the backward pass returns dL/dA through mfeast_dsy_adjoint (precision 0: FP64
    factorizations, 1: FP32 factorizations with FP64 refinement)."""
    global _FEAST_EIGH
    if _FEAST_EIGH is None:
        _FEAST_EIGH = _feast_eigh_class()
    return _FEAST_EIGH.apply(A, emin, emax, m0, fpm, precision, handle)


def feast_batched(As, emins, emaxs, m0s, fpm=None, handle=None, Bs=None):
    """Many independent real symmetric problems in one mfeast_dsygv_batched call.

    As: list of float64 GPU tensors (n_p x n_p, symmetric); Bs: None (B = I) or a list of
    symmetric positive definite float64 GPU tensors of the same sizes.  Returns the most
    significant info, a list of dicts (info, M, m0, loop, epsout, E, X, res) and the batch
    wall time (handle timing)."""
    import torch
    lib = _load()
    P = len(As)
    fpm = mfeast_init() if fpm is None else _fpm_array(fpm).copy()
    Ac = [colmajor(A.to(torch.float64)) for A in As]
    n = np.array([A.shape[0] for A in As], dtype=np.int64)
    lda = np.array([ld for _, ld in Ac], dtype=np.int64)
    m0 = np.array(m0s, dtype=np.int32)
    dev = As[0].device
    E = [torch.zeros(int(m), dtype=torch.float64, device=dev) for m in m0]
    X = [torch.zeros((int(m), int(k)), dtype=torch.float64, device=dev).mT for m, k in zip(m0, n)]
    R = [torch.zeros(int(m), dtype=torch.float64, device=dev) for m in m0]
    ptrs = lambda ts: (ctypes.c_void_p * P)(*[t.data_ptr() for t in ts])  # noqa: E731
    Ap = (ctypes.c_void_p * P)(*[a.data_ptr() for a, _ in Ac])
    Bc = None if Bs is None else [colmajor(B.to(torch.float64)) for B in Bs]
    Bp = None if Bc is None else (ctypes.c_void_p * P)(*[b.data_ptr() for b, _ in Bc])
    ldb = None if Bc is None else np.array([ld for _, ld in Bc], dtype=np.int64)
    emin = np.ascontiguousarray(np.asarray(emins, dtype=np.float64))
    emax = np.ascontiguousarray(np.asarray(emaxs, dtype=np.float64))
    M = np.zeros(P, dtype=np.int32)
    eps = np.zeros(P, dtype=np.float64)
    loop = np.zeros(P, dtype=np.int32)
    info = np.zeros(P, dtype=np.int32)
    own = handle is None
    h = Handle(dev.index or 0) if own else handle
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    dp = ctypes.POINTER(ctypes.c_double)
    try:
        ret = lib.mfeast_dsygv_batched(
            h.ptr, P, n.ctypes.data_as(i64p), Ap, lda.ctypes.data_as(i64p), Bp,
            None if ldb is None else ldb.ctypes.data_as(i64p),
            fpm.ctypes.data_as(i32p), emin.ctypes.data_as(dp), emax.ctypes.data_as(dp), m0.ctypes.data_as(i32p),
            ptrs(E), ptrs(X), n.ctypes.data_as(i64p), M.ctypes.data_as(i32p), ptrs(R), eps.ctypes.data_as(dp),
            loop.ctypes.data_as(i32p), info.ctypes.data_as(i32p))
        seconds = h.timing()[5]
    finally:
        if own:
            h.close()
    out = []
    for p in range(P):
        m = int(m0[p])
        out.append({"info": int(info[p]), "M": int(M[p]), "m0": m, "loop": int(loop[p]), "epsout": float(eps[p]),
                    "E": E[p][:m], "X": X[p][:, :m], "res": R[p][:m]})
    return int(ret), out, seconds


def mfeast_zgegv(h, n, A, lda, B, ldb, fpm, emid, r, m0, E, X, ldx, res, zne=None, wne=None):
    """C mfeast_zgegv; A, B, E, X, res device tensors (complex128 column-major A, B, X;
    E complex128 of m0 values; res float64 of m0 or 2 m0 values)."""
    lib = _load()
    fpm_a = _fpm_array(fpm)
    m0_c = ctypes.c_int32(int(m0))
    M_c = ctypes.c_int32(0)
    eps_c = ctypes.c_double(0.0)
    loop_c = ctypes.c_int32(0)
    em = np.array([complex(emid).real, complex(emid).imag], dtype=np.float64)
    zb = wb = None
    if zne is not None:
        zb = np.ascontiguousarray(np.asarray(zne, dtype=np.complex128)).view(np.float64)
        wb = np.ascontiguousarray(np.asarray(wne, dtype=np.complex128)).view(np.float64)
    hp = h.ptr if isinstance(h, Handle) else h
    info = lib.mfeast_zgegv(hp, int(n), _ptr(A), int(lda), _ptr(B), int(ldb),
                            fpm_a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(eps_c),
                            ctypes.byref(loop_c), em.ctypes.data, float(r), ctypes.byref(m0_c), _ptr(E), _ptr(X),
                            int(ldx), ctypes.byref(M_c), _ptr(res), None if zb is None else zb.ctypes.data,
                            None if wb is None else wb.ctypes.data)
    return {"info": int(info), "m0": int(m0_c.value), "M": int(M_c.value), "epsout": float(eps_c.value),
            "loop": int(loop_c.value)}


def mfeast_zgepev(h, p, n, A, lda, fpm, emid, r, m0, E, X, ldx, res, zne=None, wne=None):
    """C mfeast_zgepev; A (the p + 1 coefficient matrices, complex128 column-major, A_k at
    k lda n), E (complex128, m0), X (complex128 column-major), res (float64, m0) device
    tensors or pointers."""
    lib = _load()
    fpm_a = _fpm_array(fpm)
    m0_c = ctypes.c_int32(int(m0))
    M_c = ctypes.c_int32(0)
    eps_c = ctypes.c_double(0.0)
    loop_c = ctypes.c_int32(0)
    em = np.array([complex(emid).real, complex(emid).imag], dtype=np.float64)
    zb = wb = None
    if zne is not None:
        zb = np.ascontiguousarray(np.asarray(zne, dtype=np.complex128)).view(np.float64)
        wb = np.ascontiguousarray(np.asarray(wne, dtype=np.complex128)).view(np.float64)
    hp = h.ptr if isinstance(h, Handle) else h
    info = lib.mfeast_zgepev(hp, int(p), int(n), _ptr(A), int(lda),
                             fpm_a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(eps_c),
                             ctypes.byref(loop_c), em.ctypes.data, float(r), ctypes.byref(m0_c), _ptr(E), _ptr(X),
                             int(ldx), ctypes.byref(M_c), _ptr(res), None if zb is None else zb.ctypes.data,
                             None if wb is None else wb.ctypes.data)
    return {"info": int(info), "m0": int(m0_c.value), "M": int(M_c.value), "epsout": float(eps_c.value),
            "loop": int(loop_c.value)}


def feast_polynomial(As, emid, r, m0, fpm=None, X0=None, handle=None, zne=None, wne=None):
    """Eigenvalues of sum_k lambda^k A_k x = 0 inside the full contour (Emid, r) and their
    right eigenvectors.  As: list of the p + 1 coefficient matrices as GPU tensors (complex128
    or real, n x n).  X0: starting vectors, n x m0.  Returns a dict with E (complex), X, res,
    M, m0, loop, epsout, info."""
    import torch
    p = len(As) - 1
    n = As[0].shape[0]
    dev = As[0].device
    fpm = mfeast_init_polynomial() if fpm is None else _fpm_array(fpm).copy()
    # A(n, n, p + 1) column-major: element (i, j) of A_k at i + j n + k n n
    A_ = torch.stack([a.to(torch.complex128).mT for a in As]).contiguous()
    X = torch.zeros((m0, n), dtype=torch.complex128, device=dev).mT
    if X0 is not None:
        X[:, :X0.shape[1]].copy_(X0.to(torch.complex128))
        fpm[4] = 1
    E = torch.zeros(m0, dtype=torch.complex128, device=dev)
    res = torch.zeros(m0, dtype=torch.float64, device=dev)
    own = handle is None
    h = Handle(dev.index or 0) if own else handle
    try:
        out = mfeast_zgepev(h, p, n, A_, n, fpm, emid, r, m0, E, X, n, res, zne, wne)
        out["timing"] = h.timing()
        if fpm[51] == 1:
            out["profile"] = h.profile()
    finally:
        if own:
            h.close()
    m = out["m0"]
    out.update(E=E[:m], X=X[:, :m], res=res[:m], fpm=fpm)
    return out


def feast_general(A, B, emid, r, m0, fpm=None, X0=None, handle=None, zne=None, wne=None):
    """Eigenvalues of A x = lambda B x inside the full contour (Emid, r) and their right
    (and, with fpm[14] = 0, left) eigenvectors.  A, B: GPU tensors (complex128 or real,
    B None means identity).  X0: starting vectors, n x m0 (one-sided) or n x 2 m0 (right,
    then left).  Returns a dict with E (complex), X (right), Y (left or None), res,
    res_left, M, m0, loop, epsout, info."""
    import torch
    n = A.shape[0]
    dev = A.device
    fpm = mfeast_init_general() if fpm is None else _fpm_array(fpm).copy()
    two = int(fpm[14]) == 0
    A_, lda = colmajor(A.to(torch.complex128))
    B_, ldb = (None, n) if B is None else colmajor(B.to(torch.complex128))
    ncol = 2 * m0 if two else m0
    X = torch.zeros((ncol, n), dtype=torch.complex128, device=dev).mT
    if X0 is not None:
        X[:, :X0.shape[1]].copy_(X0.to(torch.complex128))
        fpm[4] = 1
    E = torch.zeros(m0, dtype=torch.complex128, device=dev)
    res = torch.zeros(ncol, dtype=torch.float64, device=dev)
    own = handle is None
    h = Handle(dev.index or 0) if own else handle
    try:
        out = mfeast_zgegv(h, n, A_, lda, B_, ldb, fpm, emid, r, m0, E, X, n, res, zne, wne)
        out["timing"] = h.timing()
        if fpm[51] == 1:
            out["profile"] = h.profile()
    finally:
        if own:
            h.close()
    m = out["m0"]
    out.update(E=E[:m], X=X[:, :m], Y=X[:, m0:m0 + m] if two else None, res=res[:m],
               res_left=res[m0:m0 + m] if two else None, fpm=fpm)
    return out
