"""Python binding of librexii (ctypes).  Argument marshalling only: every step
of the computation runs in the library's HIP kernels; PyTorch supplies the
device memory and the stream.

Loading fails loudly (``RuntimeError``) if ``librexii.so`` has not been built;
there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librexii.so")

PREC_FP64 = 0
PREC_MIXED = 1

STATUS = {
    0: "REXII_OK", -1: "REXII_ERR_INVALID_ARG", -2: "REXII_ERR_NONFINITE",
    -3: "REXII_ERR_NOT_CONVERGED", -4: "REXII_ERR_BREAKDOWN", -5: "REXII_ERR_OOM",
    -6: "REXII_ERR_HIP", -7: "REXII_ERR_WORKSPACE",
}


class RexiiError(RuntimeError):
    def __init__(self, status, msg, report=None):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.report = report


class SweOp(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("g", ctypes.c_double),
                ("f_cor", ctypes.c_double), ("H0", ctypes.c_double), ("H_field", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("tol", ctypes.c_double), ("precision", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("m0", ctypes.c_int32), ("rho", ctypes.c_double),
                ("pole_batch", ctypes.c_int32), ("pair_conjugate", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("method", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("scheme", ctypes.c_int32), ("reserved_opts", ctypes.c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("P", ctypes.c_int32), ("M", ctypes.c_int32), ("N", ctypes.c_int32),
                ("m0", ctypes.c_int32), ("solves", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("not_converged", ctypes.c_int32),
                ("total_iters", ctypes.c_int64), ("h", ctypes.c_double), ("t", ctypes.c_double),
                ("rho", ctypes.c_double), ("kappa_sum", ctypes.c_double),
                ("pole_tol", ctypes.c_double), ("max_rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("alg_bytes", ctypes.c_double),
                ("stagnated", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("kernel_launches", ctypes.c_int64), ("kernel_ms", ctypes.c_double),
                ("kernel_bytes", ctypes.c_double), ("step_ms", ctypes.c_double * 6),
                ("u1_bytes", ctypes.c_double), ("tile_rows", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("err_bound", ctypes.c_double), ("seconds_solve", ctypes.c_double),
                ("retried", ctypes.c_int32), ("hist_buckets", ctypes.c_int32), ("iter_hist", ctypes.c_int32 * 20)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["step_ms"] = list(d["step_ms"])
        d["iter_hist"] = list(d["iter_hist"])
        return d


EXPORTS = ["rexii_default_opts", "rexii_coeffs", "rexii_rho", "rexii_workspace_size",
           "rexii_apply", "rexii_apply_adjoint", "rexii_apply_batched", "rexii_batched_workspace_size",
           "rexii_shifted_solve", "rexii_apply_fourier", "rexii_fourier_workspace_size",
           "rexii_apply_multishift", "rexii_multishift_workspace_size", "rexii_coeffs_rexi",
           "rexii_apply_fourier_noalloc", "rexii_apply_circulant", "rexii_circulant_workspace_size",
           "rexii_fit_gaussian", "rexii_last_error"]

_lib = None


def load():
    """Load librexii.so and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2008_11607_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    lib.rexii_default_opts.argtypes = [P(Opts)]
    lib.rexii_default_opts.restype = None
    lib.rexii_coeffs.argtypes = [dbl, dbl, dbl, dbl, i32, P(i32), vp, vp, P(dbl)]
    lib.rexii_coeffs.restype = ctypes.c_int
    lib.rexii_coeffs_rexi.argtypes = [dbl, dbl, dbl, dbl, i32, P(i32), vp, vp]
    lib.rexii_coeffs_rexi.restype = ctypes.c_int
    lib.rexii_rho.argtypes = [P(SweOp), vp, P(dbl)]
    lib.rexii_rho.restype = ctypes.c_int
    lib.rexii_workspace_size.argtypes = [P(SweOp), P(Opts), dbl, P(sz)]
    lib.rexii_workspace_size.restype = ctypes.c_int
    lib.rexii_apply.argtypes = [P(SweOp), vp, vp, dbl, P(Opts), vp, sz, vp, P(Report)]
    lib.rexii_apply.restype = ctypes.c_int
    lib.rexii_apply_adjoint.argtypes = [P(SweOp), vp, vp, vp, P(dbl), dbl, P(Opts), vp, sz, vp, P(Report)]
    lib.rexii_apply_adjoint.restype = ctypes.c_int
    lib.rexii_apply_batched.argtypes = [i32, P(SweOp), P(vp), P(vp), P(dbl), P(Opts), vp, sz, vp, P(Report)]
    lib.rexii_apply_batched.restype = ctypes.c_int
    lib.rexii_batched_workspace_size.argtypes = [i32, P(SweOp), P(dbl), P(Opts), P(sz)]
    lib.rexii_batched_workspace_size.restype = ctypes.c_int
    lib.rexii_shifted_solve.argtypes = [P(SweOp), vp, dbl, i32, vp, vp, P(Opts), vp, sz, vp, P(Report)]
    lib.rexii_shifted_solve.restype = ctypes.c_int
    lib.rexii_apply_fourier.argtypes = [P(SweOp), vp, vp, dbl, i32, P(Opts), vp, sz, vp, P(Report)]
    lib.rexii_apply_fourier.restype = ctypes.c_int
    lib.rexii_apply_fourier_noalloc.argtypes = [P(SweOp), vp, vp, dbl, i32, P(Opts), vp, P(Report)]
    lib.rexii_apply_fourier_noalloc.restype = ctypes.c_int
    lib.rexii_fourier_workspace_size.argtypes = [P(SweOp), P(Opts), dbl, i32, P(sz)]
    lib.rexii_fourier_workspace_size.restype = ctypes.c_int
    lib.rexii_apply_multishift.argtypes = [P(SweOp), i32, vp, vp, dbl, P(Opts), vp, sz, vp, P(Report)]
    lib.rexii_apply_multishift.restype = ctypes.c_int
    lib.rexii_multishift_workspace_size.argtypes = [P(SweOp), i32, P(Opts), P(sz)]
    lib.rexii_multishift_workspace_size.restype = ctypes.c_int
    lib.rexii_circulant_workspace_size.argtypes = [i32, i32, vp, vp, i32, dbl, dbl, i32, i32, P(Opts), P(sz)]
    lib.rexii_circulant_workspace_size.restype = ctypes.c_int
    lib.rexii_apply_circulant.argtypes = [i32, i32, vp, vp, i32, vp, vp, dbl, dbl, i32, i32, P(Opts), vp, sz, vp,
                                          P(Report)]
    lib.rexii_apply_circulant.restype = ctypes.c_int
    lib.rexii_fit_gaussian.argtypes = [i32, dbl, dbl, i32, i32, vp, vp, P(dbl)]
    lib.rexii_fit_gaussian.restype = ctypes.c_int
    lib.rexii_last_error.argtypes = []
    lib.rexii_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def last_error():
    return load().rexii_last_error().decode()


def _check(st, report=None):
    """Raise RexiiError for a non-zero status; report: a Report, a list of
    them or a dict (converted only when raising)."""
    if st != 0:
        if isinstance(report, Report):
            report = report.as_dict()
        elif isinstance(report, list):
            report = [r.as_dict() if isinstance(r, Report) else r for r in report]
        raise RexiiError(st, last_error(), report)


def make_opts(h=None, tol=None, precision="fp64", max_iter=None, m0=None, rho=None,
              pole_batch=None, pair_conjugate=None, inner_tol=None, profile=None, method=None,
              tile_rows=None, scheme=None):
    o = Opts()
    load().rexii_default_opts(ctypes.byref(o))
    if h is not None:
        o.h = h
    if precision in ("mixed", PREC_MIXED):
        o.precision = PREC_MIXED
    elif precision in ("fp64", PREC_FP64):
        o.precision = PREC_FP64
    else:
        raise ValueError(precision)
    if tol is not None:
        o.tol = tol
    if max_iter is not None:
        o.max_iter = max_iter
    if m0 is not None:
        o.m0 = m0
    if rho is not None:
        o.rho = rho
    if pole_batch is not None:
        o.pole_batch = pole_batch
    if pair_conjugate is not None:
        o.pair_conjugate = int(pair_conjugate)
    if inner_tol is not None:
        o.inner_tol = inner_tol
    if profile is not None:
        o.profile = int(profile)
    if method is not None:
        o.method = {"auto": 0, "cocg": 0, "bicgstab": 1, "precond": 2}.get(method, method)
    if tile_rows is not None:
        o.tile_rows = int(tile_rows)
    if scheme is not None:
        o.scheme = {"rexii": 0, "rexi": 1}.get(scheme, scheme)
    return o


def make_op(nx, ny, g=1.0, fc=10.0, H=1.0, Hfield=None):
    op = SweOp()
    op.nx, op.ny, op.g, op.f_cor, op.H0 = int(nx), int(ny), float(g), float(fc), float(H)
    if Hfield is not None:
        _dev_f64(Hfield, (int(ny), int(nx)))
    op.H_field = None if Hfield is None else ctypes.c_void_p(Hfield.data_ptr())
    return op


def coeffs(t, rho, h=0.5, tol=1e-10, m0=-1):
    """(beta, alpha, kappa_sum): complex numpy arrays of the P poles and
    weights of exp(tA) ~ Re sum alpha_k (A - beta_k)^{-1} (host, FP64)."""
    lib = load()
    P = ctypes.c_int32()
    _check(lib.rexii_coeffs(t, rho, h, tol, m0, ctypes.byref(P), None, None, None))
    beta = np.zeros(2 * P.value)
    alpha = np.zeros(2 * P.value)
    kap = ctypes.c_double()
    _check(lib.rexii_coeffs(t, rho, h, tol, m0, ctypes.byref(P), beta.ctypes.data_as(ctypes.c_void_p),
                            alpha.ctypes.data_as(ctypes.c_void_p), ctypes.byref(kap)))
    return beta[0::2] + 1j * beta[1::2], alpha[0::2] + 1j * alpha[1::2], kap.value


def coeffs_rexi(t, rho, h=0.5, tol=1e-10, m0=-1):
    """(beta, alpha): complex numpy arrays of the 2N + 1 poles and weights of
    the original REXI matrix scheme, exp(tA) ~ Re sum alpha_k (A - beta_k)^{-1}."""
    lib = load()
    P = ctypes.c_int32()
    _check(lib.rexii_coeffs_rexi(t, rho, h, tol, m0, ctypes.byref(P), None, None))
    beta = np.zeros(2 * P.value)
    alpha = np.zeros(2 * P.value)
    _check(lib.rexii_coeffs_rexi(t, rho, h, tol, m0, ctypes.byref(P), beta.ctypes.data_as(ctypes.c_void_p),
                                 alpha.ctypes.data_as(ctypes.c_void_p)))
    return beta[0::2] + 1j * beta[1::2], alpha[0::2] + 1j * alpha[1::2]


def rho(nx, ny, g=1.0, fc=10.0, H=1.0, Hfield=None):
    lib = load()
    op = make_op(nx, ny, g, fc, H, Hfield)
    out = ctypes.c_double()
    _check(lib.rexii_rho(ctypes.byref(op), _stream(), ctypes.byref(out)))
    return out.value


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f64(x, shape=None):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    if shape is not None and tuple(x.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(x.shape)}")
    return x


def apply(f, t, g=1.0, fc=10.0, H=1.0, Hfield=None, out=None, **opts):
    """u = exp(tA) f on the GPU.  f: float64 CUDA tensor [3, ny, nx].
    Returns (u, report_dict)."""
    import torch
    lib = load()
    _dev_f64(f)
    ny, nx = f.shape[1], f.shape[2]
    if Hfield is not None:
        _dev_f64(Hfield, (ny, nx))
    u = torch.empty_like(f) if out is None else _dev_f64(out, f.shape)
    op = make_op(nx, ny, g, fc, H, Hfield)
    o = make_opts(**opts)
    rep = Report()
    ws = _workspace((SweOp * 1)(op), (ctypes.c_double * 1)(float(t)), o, f.device)
    st = lib.rexii_apply(ctypes.byref(op), ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                         float(t), ctypes.byref(o), *_ws_args(ws), _stream(), ctypes.byref(rep))
    _check(st, rep)
    return u, rep.as_dict()


def _workspace(ops, ts, o, device):
    """Device workspace of a slot-engine call, from PyTorch's allocator (its
    cache hands back the same memory on the next call, so repeated calls make
    no device allocation)."""
    import torch
    nb = ctypes.c_size_t()
    _check(load().rexii_batched_workspace_size(len(ops), ops, ts, ctypes.byref(o), ctypes.byref(nb)))
    if nb.value == 0:
        return None
    return torch.empty(nb.value, dtype=torch.uint8, device=device)


def _ws_args(ws):
    return (None, 0) if ws is None else (ctypes.c_void_p(ws.data_ptr()), ws.numel())


def batched_workspace_size(shapes, ts, g=1.0, fc=10.0, H=1.0, **opts):
    """Workspace bytes of apply_batched for states of the given (ny, nx)
    shapes and times (constant depth)."""
    cnt = len(shapes)
    ops = (SweOp * cnt)()
    for i, (ny, nx) in enumerate(shapes):
        ops[i] = make_op(nx, ny, g, fc, H, None)
    o = make_opts(**opts)
    nb = ctypes.c_size_t()
    _check(load().rexii_batched_workspace_size(cnt, ops, (ctypes.c_double * cnt)(*[float(t) for t in ts]),
                                               ctypes.byref(o), ctypes.byref(nb)))
    return nb.value


def shifted_solve(f, t, z, g=1.0, fc=10.0, H=1.0, Hfield=None, **opts):
    """x_k = (tA - z_k I)^{-1} f for complex shifts z (host array).
    Returns (x: complex128 CUDA tensor [npoles, 3, ny, nx], report)."""
    import torch
    lib = load()
    _dev_f64(f)
    ny, nx = f.shape[1], f.shape[2]
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    zz = np.ascontiguousarray(np.stack([z.real, z.imag], axis=1).ravel())
    x = torch.empty((len(z), 3, ny, nx), dtype=torch.complex128, device=f.device)
    op = make_op(nx, ny, g, fc, H, Hfield)
    o = make_opts(**opts)
    rep = Report()
    st = lib.rexii_shifted_solve(ctypes.byref(op), ctypes.c_void_p(f.data_ptr()), float(t), len(z),
                                 zz.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(x.data_ptr()),
                                 ctypes.byref(o), None, 0, _stream(), ctypes.byref(rep))
    _check(st, rep)
    return x, rep.as_dict()


DERIVATIVES = {"centred": 0, "spectral": 1}


def apply_fourier(f, t, g=1.0, fc=10.0, H=1.0, derivative="centred", out=None, workspace=None, **opts):
    """u = exp(tA) f by the Fourier-space path (constant depth): FFT, the
    REXII pole sum per mode in closed form, inverse FFT; FP64.
    derivative: "centred" (the operator of apply) or "spectral" (Fourier
    differentiation).  workspace: optional uint8 CUDA tensor of at least
    fourier_workspace_size() bytes (by default one from PyTorch's caching
    allocator).  Returns (u, report_dict)."""
    import torch
    lib = load()
    _dev_f64(f)
    ny, nx = f.shape[1], f.shape[2]
    u = torch.empty_like(f) if out is None else _dev_f64(out, f.shape)
    op = make_op(nx, ny, g, fc, H, None)
    o = make_opts(**opts)
    rep = Report()
    if workspace is None:
        # from PyTorch's caching allocator: repeated calls allocate nothing
        nb = ctypes.c_size_t()
        _check(lib.rexii_fourier_workspace_size(ctypes.byref(op), ctypes.byref(o), float(t),
                                                DERIVATIVES.get(derivative, derivative), ctypes.byref(nb)))
        workspace = torch.empty(nb.value, dtype=torch.uint8, device=f.device) if nb.value else None
    ws, nws = (None, 0) if workspace is None else (ctypes.c_void_p(workspace.data_ptr()), workspace.numel())
    st = lib.rexii_apply_fourier(ctypes.byref(op), ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                 float(t), DERIVATIVES.get(derivative, derivative), ctypes.byref(o), ws, nws,
                                 _stream(), ctypes.byref(rep))
    _check(st, rep)
    return u, rep.as_dict()


def apply_fourier_noalloc(f, t, g=1.0, fc=10.0, H=1.0, derivative="centred", out=None, **opts):
    """apply_fourier through rexii_apply_fourier_noalloc: the library's static
    device scratch instead of a workspace, no device allocation inside the
    call.  The grid's FFT plans must exist (fourier_workspace_size creates
    them).  out: the result tensor (allocated here when None).  Returns
    (u, report_dict)."""
    import torch
    lib = load()
    _dev_f64(f)
    ny, nx = f.shape[1], f.shape[2]
    u = torch.empty_like(f) if out is None else _dev_f64(out, f.shape)
    op = make_op(nx, ny, g, fc, H, None)
    o = make_opts(**opts)
    rep = Report()
    st = lib.rexii_apply_fourier_noalloc(ctypes.byref(op), ctypes.c_void_p(f.data_ptr()),
                                         ctypes.c_void_p(u.data_ptr()), float(t),
                                         DERIVATIVES.get(derivative, derivative), ctypes.byref(o), _stream(),
                                         ctypes.byref(rep))
    _check(st, rep)
    return u, rep.as_dict()


STATIC_SCRATCH_BYTES = 256 << 20


def apply_multishift(f, t, g=1.0, fc=10.0, H=1.0, Hfield=None, out=None, **opts):
    """u = exp(tA) f by the shared-Krylov (multi-shift) path: one W-skew
    Lanczos process per state serves every pole; FP64, any depth.
    f: float64 CUDA tensor [3, ny, nx] or a batch [nrhs, 3, ny, nx] sharing
    the operator and t.  Returns (u, report_dict)."""
    import torch
    lib = load()
    _dev_f64(f)
    if f.dim() not in (3, 4) or f.shape[-3] != 3:
        raise ValueError("expected [3, ny, nx] or [nrhs, 3, ny, nx]")
    nrhs = 1 if f.dim() == 3 else f.shape[0]
    ny, nx = f.shape[-2], f.shape[-1]
    if Hfield is not None:
        _dev_f64(Hfield, (ny, nx))
    u = torch.empty_like(f) if out is None else _dev_f64(out, f.shape)
    op = make_op(nx, ny, g, fc, H, Hfield)
    o = make_opts(**opts)
    rep = Report()
    nb = ctypes.c_size_t()
    _check(lib.rexii_multishift_workspace_size(ctypes.byref(op), int(nrhs), ctypes.byref(o), ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=f.device) if nb.value else None
    st = lib.rexii_apply_multishift(ctypes.byref(op), int(nrhs), ctypes.c_void_p(f.data_ptr()),
                                    ctypes.c_void_p(u.data_ptr()), float(t), ctypes.byref(o), *_ws_args(ws),
                                    _stream(), ctypes.byref(rep))
    _check(st, rep)
    return u, rep.as_dict()


def fourier_workspace_size(nx, ny, t, g=1.0, fc=10.0, H=1.0, derivative="centred", **opts):
    lib = load()
    op = make_op(nx, ny, g, fc, H, None)
    o = make_opts(**opts)
    out = ctypes.c_size_t()
    _check(lib.rexii_fourier_workspace_size(ctypes.byref(op), ctypes.byref(o), float(t),
                                            DERIVATIVES.get(derivative, derivative), ctypes.byref(out)))
    return out.value


def workspace_size(nx, ny, t, g=1.0, fc=10.0, H=1.0, **opts):
    lib = load()
    op = make_op(nx, ny, g, fc, H, None)
    o = make_opts(**opts)
    out = ctypes.c_size_t()
    _check(lib.rexii_workspace_size(ctypes.byref(op), ctypes.byref(o), float(t), ctypes.byref(out)))
    return out.value


def apply_adjoint(f, gbar, t, g=1.0, fc=10.0, H=1.0, want_dJdf=True, want_dJdH=True, **opts):
    """Reverse mode of apply for a loss J(u): gbar = dJ/du (float64 CUDA
    [3, ny, nx]).  Returns (dJdf tensor or None, dJdH float or None, report).
    The pole set is the one apply uses for (t, H) and is held fixed."""
    import torch
    lib = load()
    _dev_f64(gbar)
    ny, nx = gbar.shape[1], gbar.shape[2]
    if f is not None:
        _dev_f64(f, gbar.shape)
    dJdf = torch.empty_like(gbar) if want_dJdf else None
    dJdH = ctypes.c_double(0.0)
    op = make_op(nx, ny, g, fc, H, None)
    o = make_opts(**opts)
    rep = Report()
    st = lib.rexii_apply_adjoint(ctypes.byref(op), ctypes.c_void_p(f.data_ptr()) if f is not None else None,
                                 ctypes.c_void_p(gbar.data_ptr()),
                                 ctypes.c_void_p(dJdf.data_ptr()) if dJdf is not None else None,
                                 ctypes.byref(dJdH) if want_dJdH else None, float(t), ctypes.byref(o), None, 0,
                                 _stream(), ctypes.byref(rep))
    _check(st, rep)
    return dJdf, (dJdH.value if want_dJdH else None), rep.as_dict()


def apply_batched(fs, ts, g=1.0, fc=10.0, H=1.0, Hfield=None, **opts):
    """u_i = exp(t_i A_i) f_i for a list of states (grids may differ) in one
    call: all problems' solves share one slot scheduler.  g, fc, H and Hfield
    (depth fields, CUDA float64 [ny, nx]) may be scalars / one tensor or
    per-problem lists.  Returns (list of u, list of reports)."""
    import torch
    lib = load()
    cnt = len(fs)

    def per(v, i):
        return v[i] if isinstance(v, (list, tuple)) else v

    ops = (SweOp * cnt)()
    us = [torch.empty_like(_dev_f64(f)) for f in fs]
    for i, f in enumerate(fs):
        ops[i] = make_op(f.shape[2], f.shape[1], per(g, i), per(fc, i), per(H, i), per(Hfield, i))
    fptr = (ctypes.c_void_p * cnt)(*[ctypes.c_void_p(f.data_ptr()) for f in fs])
    uptr = (ctypes.c_void_p * cnt)(*[ctypes.c_void_p(u.data_ptr()) for u in us])
    tarr = (ctypes.c_double * cnt)(*[float(t) for t in ts])
    reps = (Report * cnt)()
    o = make_opts(**opts)
    ws = _workspace(ops, tarr, o, fs[0].device)
    st = lib.rexii_apply_batched(cnt, ops, fptr, uptr, tarr, ctypes.byref(o), *_ws_args(ws), _stream(), reps)
    _check(st, list(reps))
    return us, [r.as_dict() for r in reps]


def fit_gaussian(L=24, mu=-5.133333333333333, x_max=60.0, K=200, n_candidates=200001):
    """Refit of the Gaussian's rational approximation (host, FP64): returns
    (a: complex numpy array a_0..a_L, points, max_err)."""
    a = np.zeros(2 * (L + 1))
    pts = np.zeros(K)
    err = ctypes.c_double()
    _check(load().rexii_fit_gaussian(int(L), float(mu), float(x_max), int(K), int(n_candidates),
                                     a.ctypes.data_as(ctypes.c_void_p), pts.ctypes.data_as(ctypes.c_void_p),
                                     ctypes.byref(err)))
    return a[0::2] + 1j * a[1::2], pts, err.value


CIRC_SCHEMES = {"rexii": 0, "rexi": 1, "rexie": 2}


def _stencil_arrays(stencil):
    off = np.ascontiguousarray(np.array(list(stencil.keys()), dtype=np.int32))
    c = np.array([complex(v) for v in stencil.values()], dtype=np.complex128)
    cc = np.ascontiguousarray(np.stack([c.real, c.imag], axis=1).ravel())
    return off, cc


def apply_circulant(f, t, stencil, scheme="rexii", nu=0.0, M=0, out=None, **opts):
    """exp(tA) f for a circulant matrix A, (A f)_j = sum_d stencil[d] f_{j+d}
    (indices mod n), by REXII, the original REXI or REXIE (scheme), each
    resolvent exact per Fourier mode on the GPU.  f: float64 CUDA tensor [n]
    or [nrhs, n] of real vectors.  nu: REXIE's shift, a purely imaginary
    number (A - nu I = i B).  M > 0 fixes M, else the rule of
    eq. matrixAccuracyBound.  Returns (u: complex128 CUDA tensor shaped like
    f, report_dict)."""
    import torch
    lib = load()
    _dev_f64(f)
    if f.dim() not in (1, 2):
        raise ValueError("expected [n] or [nrhs, n]")
    nrhs = 1 if f.dim() == 1 else f.shape[0]
    n = f.shape[-1]
    nu = complex(nu)
    if nu.real != 0.0:
        raise ValueError("nu must be purely imaginary")
    u = torch.empty(f.shape, dtype=torch.complex128, device=f.device) if out is None else out
    if not (u.is_cuda and u.dtype == torch.complex128 and u.is_contiguous() and u.shape == f.shape):
        raise ValueError("out must be a contiguous complex128 CUDA tensor shaped like f")
    off, cc = _stencil_arrays(stencil)
    o = make_opts(**opts)
    rep = Report()
    nb = ctypes.c_size_t()
    _check(lib.rexii_circulant_workspace_size(int(n), len(off), off.ctypes.data_as(ctypes.c_void_p),
                                              cc.ctypes.data_as(ctypes.c_void_p), int(nrhs), float(t), float(nu.imag),
                                              CIRC_SCHEMES.get(scheme, scheme), int(M), ctypes.byref(o),
                                              ctypes.byref(nb)))
    ws = torch.empty(nb.value, dtype=torch.uint8, device=f.device) if nb.value else None
    st = lib.rexii_apply_circulant(int(n), len(off), off.ctypes.data_as(ctypes.c_void_p),
                                   cc.ctypes.data_as(ctypes.c_void_p), int(nrhs), ctypes.c_void_p(f.data_ptr()),
                                   ctypes.c_void_p(u.data_ptr()), float(t), float(nu.imag),
                                   CIRC_SCHEMES.get(scheme, scheme), int(M), ctypes.byref(o), *_ws_args(ws),
                                   _stream(), ctypes.byref(rep))
    _check(st, rep)
    return u, rep.as_dict()


def circulant_workspace_size(n, t, stencil, nrhs=1, scheme="rexii", nu=0.0, M=0, **opts):
    lib = load()
    off, cc = _stencil_arrays(stencil)
    o = make_opts(**opts)
    out = ctypes.c_size_t()
    _check(lib.rexii_circulant_workspace_size(int(n), len(off), off.ctypes.data_as(ctypes.c_void_p),
                                              cc.ctypes.data_as(ctypes.c_void_p), int(nrhs), float(t),
                                              float(complex(nu).imag), CIRC_SCHEMES.get(scheme, scheme), int(M),
                                              ctypes.byref(o), ctypes.byref(out)))
    return out.value


def _autograd_fn():
    import torch

    class RexiiExp(torch.autograd.Function):
        """u = exp(tA(H)) f with gradients w.r.t. f and the constant depth H
        (a 0-d float64 tensor).  The pole set is frozen at the forward call
        (its rho is taken at the given H), so the gradient is that of the
        fixed rational approximation."""

        @staticmethod
        def forward(ctx, f, H, t, g, fc, opts):
            Hv = float(H)
            rho = opts.get("rho") or globals()["rho"](f.shape[2], f.shape[1], g=g, fc=fc, H=Hv)
            o = dict(opts)
            o["rho"] = rho
            u, _ = apply(f.contiguous(), t, g=g, fc=fc, H=Hv, **o)
            ctx.save_for_backward(f)
            ctx.args = (Hv, t, g, fc, o)
            return u

        @staticmethod
        def backward(ctx, gu):
            (f,) = ctx.saved_tensors
            Hv, t, g, fc, o = ctx.args
            need_f, need_H = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            dJdf, dJdH, _ = apply_adjoint(f.contiguous(), gu.contiguous(), t, g=g, fc=fc, H=Hv,
                                          want_dJdf=need_f, want_dJdH=need_H, **o)
            gH = torch.tensor(dJdH, dtype=torch.float64, device=f.device) if need_H else None
            return dJdf, gH, None, None, None, None

    return RexiiExp


_RexiiExp = None


def rexii_exp(f, H, t, g=1.0, fc=10.0, **opts):
    """Differentiable u = exp(t A(H)) f (see RexiiExp)."""
    global _RexiiExp
    if _RexiiExp is None:
        _RexiiExp = _autograd_fn()
    return _RexiiExp.apply(f, H, t, g, fc, opts)
