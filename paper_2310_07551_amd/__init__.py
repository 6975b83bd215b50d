"""split-ETD3 on MI355X: Python binding of libsetd (include/setd.h).

Argument marshalling only.  torch supplies device memory and the current HIP
stream; every computation runs in the library's HIP kernels.  Tensors are
flat FP64 CUDA (ROCm) tensors in the layout of setd.h: index i_1 fastest
(a torch tensor of shape (n_d, ..., n_1) in torch's row-major order has that
layout), matrices column-major (pass M.T.contiguous() of a row-major torch
matrix, or use `colmajor`).
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

from . import _lib
from ._lib import (G_FHN, G_NONE, G_SCHNAKENBERG, PREC_BF16X2, PREC_BF16X3, PREC_F32, PREC_F64, PREC_I8X4, STAGE_2, STAGE_3,
                   STAGE_F, SetdError)

__all__ = [
    "phi_matrices", "tucker_apply", "tucker_apply_noalloc", "Context", "Batch", "field_norms", "profile_enable", "profile_read", "colmajor", "version", "SetdError",
    "G_NONE", "G_SCHNAKENBERG", "G_FHN", "PREC_F64", "PREC_F32", "PREC_BF16X3", "PREC_BF16X2", "PREC_I8X4", "STAGE_2", "STAGE_3",
    "STAGE_F",
]


def _torch():
    import torch
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _check_dev(t, what: str, dtype=None):
    torch = _torch()
    dtype = torch.float64 if dtype is None else dtype
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU tensor" % what)
    if t.dtype != dtype:
        raise TypeError("%s must have dtype %s" % (what, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)


def colmajor(M):
    """A row-major torch matrix -> contiguous tensor holding it column-major."""
    return M.t().contiguous()


def version() -> str:
    return _lib.load().setd_version().decode()


def phi_matrices(A, tau: float, ell: int, stream=None):
    """phi_0(tau A), ..., phi_ell(tau A) for a column-major n x n FP64 matrix A
    (flat or (n, n) tensor holding column-major data).  Returns a tensor of
    shape (ell + 1, n * n), each row a column-major matrix."""
    torch = _torch()
    _check_dev(A, "A")
    n = int(round(A.numel() ** 0.5))
    if n * n != A.numel():
        raise ValueError("A must hold n*n values")
    out = torch.empty((ell + 1, n * n), dtype=torch.float64, device=A.device)
    lib = _lib.load()
    _lib.check(lib.setd_phi_matrices(A.data_ptr(), n, float(tau), int(ell), out.data_ptr(), _stream(stream)))
    return out


def tucker_apply(V, W, dims: Sequence[int], mats: Sequence[Optional[object]], alpha: float = 1.0,
                 beta: float = 0.0, prec: int = PREC_F64, workspace=None, stream=None):
    """W <- alpha * (V x_1 M_1 ... x_d M_d) + beta * W (in place on W).
    mats[mu] is a column-major n_mu x n_mu FP64 tensor or None (identity)."""
    _check_dev(V, "V")
    _check_dev(W, "W")
    d = len(dims)
    cdims = (ctypes.c_int64 * d)(*[int(x) for x in dims])
    ptrs = (ctypes.c_void_p * d)()
    for mu, M in enumerate(mats):
        if M is None:
            ptrs[mu] = None
        else:
            _check_dev(M, "M[%d]" % mu)
            ptrs[mu] = M.data_ptr()
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        _check_dev(workspace, "workspace", dtype=workspace.dtype)
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    lib = _lib.load()
    _lib.check(lib.setd_tucker_apply(V.data_ptr(), W.data_ptr(), d, cdims, ptrs, float(alpha), float(beta),
                                     int(prec), ws_ptr, ws_bytes, _stream(stream)))
    return W


def tucker_apply_noalloc(V, W, dims: Sequence[int], mats: Sequence[Optional[object]], alpha: float = 1.0,
                         beta: float = 0.0, prec: int = PREC_F64, stream=None):
    """tucker_apply through setd_tucker_apply_noalloc: no device allocation,
    the library's per-GPU scratch array (NOALLOC_SCRATCH_BYTES) as workspace."""
    _check_dev(V, "V")
    _check_dev(W, "W")
    d = len(dims)
    cdims = (ctypes.c_int64 * d)(*[int(x) for x in dims])
    ptrs = (ctypes.c_void_p * d)()
    for mu, M in enumerate(mats):
        if M is None:
            ptrs[mu] = None
        else:
            _check_dev(M, "M[%d]" % mu)
            ptrs[mu] = M.data_ptr()
    _lib.check(_lib.load().setd_tucker_apply_noalloc(V.data_ptr(), W.data_ptr(), d, cdims, ptrs, float(alpha),
                                                     float(beta), int(prec), _stream(stream)))
    return W


def tucker_workspace_bytes(dims: Sequence[int], prec: int = PREC_F64) -> int:
    d = len(dims)
    cdims = (ctypes.c_int64 * d)(*[int(x) for x in dims])
    return int(_lib.load().setd_tucker_workspace_bytes(d, cdims, int(prec)))


def field_norms(x, y=None, stream=None):
    """(||x||_2, ||x||_inf, ||x-y||_2, ||x-y||_inf) with deterministic reductions."""
    _check_dev(x, "x")
    if y is not None:
        _check_dev(y, "y")
        if y.numel() != x.numel():
            raise ValueError("x and y differ in size")
    out = (ctypes.c_double * 4)()
    _lib.check(_lib.load().setd_field_norms(x.data_ptr(), None if y is None else y.data_ptr(), x.numel(), out,
                                            _stream(stream)))
    return tuple(out)


def profile_enable(on: bool = True):
    """Bracket every library kernel launch with HIP events (see setd.h)."""
    _lib.check(_lib.load().setd_profile_enable(1 if on else 0))


def profile_read(reset: bool = True) -> dict:
    """{class: {"launches", "ms", "flops", "bytes"}} since the last reset."""
    n = len(_lib.PROF_CLASSES)
    out = (ctypes.c_double * (4 * n))()
    _lib.check(_lib.load().setd_profile_read(out, 1 if reset else 0))
    return {name: dict(launches=int(out[4 * k]), ms=out[4 * k + 1], flops=out[4 * k + 2], bytes=out[4 * k + 3])
            for k, name in enumerate(_lib.PROF_CLASSES)}


class Context:
    """An integration context (setd_ctx): grid, matrices A_mu^(c), tau, arithmetic."""

    def __init__(self, dims: Sequence[int], A: Sequence[Sequence[object]], tau: float, prec: int = PREC_F64,
                 stream=None):
        self.dims = tuple(int(x) for x in dims)
        self.d = len(self.dims)
        self.ncomp = len(A)
        self.tau = float(tau)
        self.prec = prec
        self.N = 1
        for x in self.dims:
            self.N *= x
        ptrs = (ctypes.c_void_p * (self.ncomp * self.d))()
        for c in range(self.ncomp):
            for mu in range(self.d):
                _check_dev(A[c][mu], "A[%d][%d]" % (c, mu))
                ptrs[c * self.d + mu] = A[c][mu].data_ptr()
        cdims = (ctypes.c_int64 * self.d)(*self.dims)
        h = ctypes.c_void_p()
        lib = _lib.load()
        _lib.check(lib.setd_ctx_create(ctypes.byref(h), self.d, cdims, self.ncomp, ptrs, self.tau, int(prec),
                                       _stream(stream)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().setd_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def split_phi_apply(self, comp: int, ell: int, stage: int, V, W, scale: float = 1.0, beta: float = 0.0,
                        stream=None):
        """W <- beta W + scale * S_ell(c_stage tau) V."""
        _check_dev(V, "V")
        _check_dev(W, "W")
        _lib.check(_lib.load().setd_split_phi_apply(self._h, comp, ell, stage, V.data_ptr(), W.data_ptr(),
                                                    float(scale), float(beta), _stream(stream)))
        return W

    def step(self, u, nsteps: int, g_kind: int, params: Sequence[float], tau: Optional[float] = None,
             stream=None):
        """Advance u (ncomp*N FP64, component-major) by nsteps split-ETD3 steps, in place."""
        _check_dev(u, "u")
        if u.numel() != self.ncomp * self.N:
            raise ValueError("u must hold ncomp*N values")
        p = (ctypes.c_double * max(1, len(params)))(*[float(x) for x in params])
        t = self.tau if tau is None else float(tau)
        _lib.check(_lib.load().setd_etd_step(self._h, u.data_ptr(), int(nsteps), t, int(g_kind), p, len(params),
                                             _stream(stream)))
        self.tau = t
        return u

    def step_cplx(self, u, nsteps: int, g_kind: int, params: Sequence[float], tau: Optional[float] = None,
                  stream=None):
        """Advance u by nsteps exprk3ds_cplx steps (complex two-term splitting), in place."""
        _check_dev(u, "u")
        if u.numel() != self.ncomp * self.N:
            raise ValueError("u must hold ncomp*N values")
        p = (ctypes.c_double * max(1, len(params)))(*[float(x) for x in params])
        t = self.tau if tau is None else float(tau)
        _lib.check(_lib.load().setd_etd_cplx_step(self._h, u.data_ptr(), int(nsteps), t, int(g_kind), p, len(params),
                                                  _stream(stream)))
        self.tau = t
        return u

    def step_record(self, u, rec, g_kind: int, params: Sequence[float], tau: Optional[float] = None,
                    stream=None):
        """One split-ETD3 step of u in place that also writes the step's stage
        quantities (G, F, U2, D2, U3, D3; 6*ncomp*N FP64) into rec, for
        adjoint_step(..., rec=rec) (setd_etd_step_record)."""
        _check_dev(u, "u")
        _check_dev(rec, "rec")
        if u.numel() != self.ncomp * self.N:
            raise ValueError("u must hold ncomp*N values")
        if rec.numel() < 6 * self.ncomp * self.N:
            raise ValueError("rec needs 6*ncomp*N values")
        p = (ctypes.c_double * max(1, len(params)))(*[float(x) for x in params])
        t = self.tau if tau is None else float(tau)
        _lib.check(_lib.load().setd_etd_step_record(self._h, u.data_ptr(), t, int(g_kind), p, len(params),
                                                    rec.data_ptr(), _stream(stream)))
        self.tau = t
        return u

    def adjoint_step(self, u, ubar, g_kind: int, params: Sequence[float], grad, sigma_mask: int = 0,
                     rec=None, stream=None):
        """One step backwards: ubar <- (dU'/dU)^T ubar at state u; grad (FP64
        device, len(params) + ncomp) accumulates the parameter and diffusion-size
        gradients (setd_etd_adjoint_step).  With rec (written by step_record
        for this u) the stage quantities are not recomputed
        (setd_etd_adjoint_step_recorded)."""
        _check_dev(u, "u")
        _check_dev(ubar, "ubar")
        _check_dev(grad, "grad")
        if u.numel() != self.ncomp * self.N or ubar.numel() != u.numel():
            raise ValueError("u and ubar must hold ncomp*N values")
        if grad.numel() < len(params) + self.ncomp:
            raise ValueError("grad needs len(params) + ncomp entries")
        p = (ctypes.c_double * max(1, len(params)))(*[float(x) for x in params])
        lib = _lib.load()
        if rec is None:
            _lib.check(lib.setd_etd_adjoint_step(self._h, u.data_ptr(), ubar.data_ptr(), int(g_kind), p, len(params),
                                                 int(sigma_mask), grad.data_ptr(), _stream(stream)))
        else:
            _check_dev(rec, "rec")
            if rec.numel() < 6 * self.ncomp * self.N:
                raise ValueError("rec needs 6*ncomp*N values")
            _lib.check(lib.setd_etd_adjoint_step_recorded(self._h, u.data_ptr(), rec.data_ptr(), ubar.data_ptr(),
                                                          int(g_kind), p, len(params), int(sigma_mask),
                                                          grad.data_ptr(), _stream(stream)))
        return ubar

    def step2(self, u, nsteps: int, g_kind: int, params: Sequence[float], tau: Optional[float] = None,
              stream=None):
        """Advance u by nsteps steps of the second-order split integrator etd2rkds, in place."""
        _check_dev(u, "u")
        if u.numel() != self.ncomp * self.N:
            raise ValueError("u must hold ncomp*N values")
        p = (ctypes.c_double * max(1, len(params)))(*[float(x) for x in params])
        t = self.tau if tau is None else float(tau)
        _lib.check(_lib.load().setd_etd2_step(self._h, u.data_ptr(), int(nsteps), t, int(g_kind), p, len(params),
                                              _stream(stream)))
        self.tau = t
        return u


class Batch:
    """Many independent instances advanced together (setd_batch).

    dims: sequence of per-instance grid sizes (each a tuple of d ints);
    A: per instance, per component, per direction a column-major FP64 device
    matrix (A[b][c][mu]).  The batch state is one flat FP64 device tensor in
    the layout given by `layout()` (see setd.h)."""

    def __init__(self, dims, A, tau: float, prec: int = PREC_F64, stream=None):
        self.dims = [tuple(int(x) for x in dm) for dm in dims]
        self.nbatch = len(self.dims)
        if self.nbatch == 0:
            raise ValueError("empty batch")
        self.d = len(self.dims[0])
        if any(len(dm) != self.d for dm in self.dims):
            raise ValueError("every instance needs the same number of dimensions")
        self.ncomp = len(A[0])
        flat = []
        for b in range(self.nbatch):
            if len(A[b]) != self.ncomp:
                raise ValueError("every instance needs the same number of components")
            for c in range(self.ncomp):
                for mu in range(self.d):
                    _check_dev(A[b][c][mu], "A[%d][%d][%d]" % (b, c, mu))
                    flat.append(A[b][c][mu].data_ptr())
        ptrs = (ctypes.c_void_p * len(flat))(*flat)
        cdims = (ctypes.c_int64 * (self.nbatch * self.d))(*[x for dm in self.dims for x in dm])
        h = ctypes.c_void_p()
        lib = _lib.load()
        _lib.check(lib.setd_batch_create(ctypes.byref(h), self.nbatch, self.d, cdims, self.ncomp, ptrs, float(tau),
                                         int(prec), _stream(stream)))
        self._h = h
        self.tau = float(tau)
        off = (ctypes.c_int64 * (self.nbatch + 1))()
        cs = (ctypes.c_int64 * self.nbatch)()
        _lib.check(lib.setd_batch_layout(self._h, off, cs))
        self.offsets = list(off)
        self.cstride = list(cs)
        self.total = self.offsets[-1]

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().setd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def field(self, u, b: int, c: int):
        """View of component c of instance b inside the flat state u (flat, N_b values)."""
        n = 1
        for x in self.dims[b]:
            n *= x
        o = self.offsets[b] + c * self.cstride[b]
        return u[o:o + n]

    def step(self, u, nsteps: int, g_kind: int, params, stream=None):
        """Advance every instance by nsteps split-ETD3 steps, in place.  params:
        one sequence of reaction parameters per instance (or one shared)."""
        _check_dev(u, "u")
        if u.numel() != self.total:
            raise ValueError("u must hold %d values (layout())" % self.total)
        params = list(params)
        if params and not hasattr(params[0], "__len__"):
            params = [params] * self.nbatch
        if len(params) not in (0, self.nbatch):
            raise ValueError("params: one entry per instance")
        npar = len(params[0]) if params else 0
        flat = [float(x) for p in params for x in p]
        if any(len(p) != npar for p in params):
            raise ValueError("every instance needs the same number of parameters")
        arr = (ctypes.c_double * max(1, len(flat)))(*flat)
        _lib.check(_lib.load().setd_batch_step(self._h, u.data_ptr(), int(nsteps), int(g_kind), arr, npar,
                                               _stream(stream)))
        return u

    def tune(self, stream=None):
        _lib.check(_lib.load().setd_batch_tune(self._h, _stream(stream)))
        return self.info()

    def set_tiles(self, mode1, modeB):
        """mode1, modeB: (tm, tn, grid_cap) each."""
        cfg = (ctypes.c_int * 6)(*[int(x) for x in tuple(mode1) + tuple(modeB)])
        _lib.check(_lib.load().setd_batch_set_tiles(self._h, cfg))

    def info(self) -> dict:
        out = (ctypes.c_int64 * _lib.BATCH_INFO)()
        _lib.check(_lib.load().setd_batch_info(self._h, out))
        return dict(mode1=tuple(out[0:3]), modeB=tuple(out[3:6]), tuned=bool(out[6]), launches_per_step=int(out[7]),
                    total=int(out[8]), packed_sets=int(out[9]))
