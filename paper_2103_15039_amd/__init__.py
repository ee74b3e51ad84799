"""Python binding of liblsgcpd, the MI355X (gfx950) LSG-CPD library.

Argument marshalling only: every step of the method runs in the HIP kernels of
liblsgcpd.so (include/lsgcpd.h).  Arrays are torch CUDA (HIP) float32 tensors;
torch provides device memory and the current stream, nothing else.  The module
raises if the shared library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsgcpd.so")

OK, E_INVALID, E_HIP, E_NOMEM, E_NUMERIC, E_UNSUPPORTED = range(6)
EXACT_NORMALIZER = 1
PAIRS_LDS = 2
PAIRS_MFMA = 4
DENSE = 8
GRAPH = 16
BF16_CROSS = 32
_BACKENDS = {"scalar": 0, "lds": PAIRS_LDS, "mfma": PAIRS_MFMA, "dense": DENSE}
NSTATS = 86

SYMBOLS = ("lsgcpd_abi_version", "lsgcpd_status_string", "lsgcpd_ctx_create",
           "lsgcpd_ctx_destroy", "lsgcpd_last_error", "lsgcpd_params_default",
           "lsgcpd_normals", "lsgcpd_estep", "lsgcpd_register", "lsgcpd_register_batch",
           "lsgcpd_depth_confidence", "lsgcpd_register_cf", "lsgcpd_autotune",
           "lsgcpd_profile_enable", "lsgcpd_profile_read", "lsgcpd_profile_launches",
           "lsgcpd_estep_noalloc", "lsgcpd_proposal_inputs", "lsgcpd_proposal_forward",
           "lsgcpd_proposal_train_step", "lsgcpd_register_proposed")
ABI_VERSION = 6


class Pose(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3)]


class EstepOut(C.Structure):
    _fields_ = [("sigma2", C.c_double), ("gamma", C.c_double), ("V", C.c_double),
                ("sumP", C.c_double), ("outlier_mass", C.c_double), ("nll", C.c_double),
                ("pd", C.c_double), ("stats", C.c_double * NSTATS), ("grad", C.c_double * 6),
                ("hess", C.c_double * 36), ("pose_next", Pose), ("sigma2_next", C.c_double),
                ("newton_iters", C.c_int32), ("gn_fallbacks", C.c_int32),
                ("bf16_cross", C.c_int32), ("pad", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("k", C.c_int32), ("alpha_max", C.c_double), ("lambda_", C.c_double),
                ("w0", C.c_double), ("V", C.c_double), ("max_iter", C.c_int32),
                ("tol", C.c_double), ("sigma2_init", C.c_double), ("newton_max", C.c_int32),
                ("flags", C.c_uint32), ("eta", C.c_double)]


class Report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("gn_fallbacks", C.c_int32),
                ("sigma2", C.c_double), ("nll_first", C.c_double), ("nll_last", C.c_double),
                ("V", C.c_double), ("w0", C.c_double), ("n_used", C.c_int64),
                ("m_used", C.c_int64), ("bf16_steps", C.c_int32), ("pad", C.c_int32)]


class Profile(C.Structure):
    _fields_ = [("launches", C.c_int64), ("pairs", C.c_int64), ("pair_kernel_ms", C.c_double),
                ("estep_ms", C.c_double), ("evaluated_pairs", C.c_int64)]


class LsgcpdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_STATUS = {OK: "LSGCPD_OK", E_INVALID: "LSGCPD_E_INVALID", E_HIP: "LSGCPD_E_HIP",
           E_NOMEM: "LSGCPD_E_NOMEM", E_NUMERIC: "LSGCPD_E_NUMERIC",
           E_UNSUPPORTED: "LSGCPD_E_UNSUPPORTED"}

_lib = None
_ctx = {}


def load_library(path=LIB_PATH):
    """Loads liblsgcpd.so and declares its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_2103_15039_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(path)
    vp, i64, i32, u32, d = C.c_void_p, C.c_int64, C.c_int32, C.c_uint32, C.c_double
    lib.lsgcpd_abi_version.restype = C.c_int
    if lib.lsgcpd_abi_version() != ABI_VERSION:
        raise ImportError(f"{path} has ABI version {lib.lsgcpd_abi_version()}, this binding "
                          f"expects {ABI_VERSION}: rebuild it")
    lib.lsgcpd_status_string.restype = C.c_char_p
    lib.lsgcpd_status_string.argtypes = [C.c_int]
    lib.lsgcpd_ctx_create.restype = C.c_int
    lib.lsgcpd_ctx_create.argtypes = [C.c_int, C.POINTER(vp)]
    lib.lsgcpd_ctx_destroy.restype = None
    lib.lsgcpd_ctx_destroy.argtypes = [vp]
    lib.lsgcpd_last_error.restype = C.c_char_p
    lib.lsgcpd_last_error.argtypes = [vp]
    lib.lsgcpd_params_default.restype = None
    lib.lsgcpd_params_default.argtypes = [C.POINTER(Params)]
    lib.lsgcpd_normals.restype = C.c_int
    lib.lsgcpd_normals.argtypes = [vp, vp, i64, i32, d, d, vp, vp, vp, vp]
    lib.lsgcpd_estep.restype = C.c_int
    lib.lsgcpd_estep.argtypes = [vp, vp, i64, vp, vp, vp, i64, vp, vp, d, d, C.POINTER(Pose), d,
                                 u32, C.POINTER(EstepOut), vp, vp, vp]
    lib.lsgcpd_estep_noalloc.restype = C.c_int
    lib.lsgcpd_estep_noalloc.argtypes = lib.lsgcpd_estep.argtypes
    lib.lsgcpd_register.restype = C.c_int
    lib.lsgcpd_register.argtypes = [vp, vp, i64, vp, i64, C.POINTER(Params), C.POINTER(Pose),
                                    C.POINTER(Pose), C.POINTER(Report), vp, vp]
    lib.lsgcpd_register_batch.restype = C.c_int
    lib.lsgcpd_register_batch.argtypes = [vp, i32, vp, vp, vp, vp, C.POINTER(Params),
                                          C.POINTER(Pose), C.POINTER(Pose), C.POINTER(Report), vp]
    lib.lsgcpd_depth_confidence.restype = C.c_int
    lib.lsgcpd_depth_confidence.argtypes = [vp, vp, i64, C.POINTER(C.c_double), d, vp, vp]
    lib.lsgcpd_register_cf.restype = C.c_int
    lib.lsgcpd_register_cf.argtypes = [vp, vp, vp, i64, vp, vp, i64, d, C.POINTER(Params),
                                       C.POINTER(Pose), C.POINTER(Pose), C.POINTER(Report), vp,
                                       vp]
    lib.lsgcpd_autotune.restype = C.c_int
    lib.lsgcpd_autotune.argtypes = [vp, vp, i64, vp, i64, C.POINTER(Params), C.POINTER(i32), vp]
    lib.lsgcpd_profile_enable.restype = C.c_int
    lib.lsgcpd_profile_enable.argtypes = [vp, C.c_int]
    lib.lsgcpd_profile_read.restype = C.c_int
    lib.lsgcpd_profile_read.argtypes = [vp, C.POINTER(Profile), C.c_int]
    lib.lsgcpd_profile_launches.restype = C.c_int
    lib.lsgcpd_profile_launches.argtypes = [vp, C.POINTER(d), C.POINTER(d), i64,
                                            C.POINTER(i64)]
    lib.lsgcpd_proposal_inputs.restype = C.c_int
    lib.lsgcpd_proposal_inputs.argtypes = [vp, i32, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp]
    lib.lsgcpd_proposal_forward.restype = C.c_int
    lib.lsgcpd_proposal_forward.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp, vp]
    lib.lsgcpd_proposal_train_step.restype = C.c_int
    lib.lsgcpd_proposal_train_step.argtypes = [vp, vp, vp, vp, i32, d, i32, i32, vp, vp, vp, i32,
                                               vp, vp, vp, vp, vp, vp]
    lib.lsgcpd_register_proposed.restype = C.c_int
    lib.lsgcpd_register_proposed.argtypes = [vp, i32, vp, vp, vp, vp, C.POINTER(Params), vp, i32,
                                             d, C.POINTER(Pose), C.POINTER(Report), vp, vp]
    _lib = lib
    return lib


def _torch():
    import torch
    return torch


def context(device=0):
    """The library context of a HIP device (created on first use)."""
    lib = load_library()
    if device not in _ctx:
        h = C.c_void_p()
        st = lib.lsgcpd_ctx_create(int(device), C.byref(h))
        if st != OK:
            raise LsgcpdError(st, f"cannot open HIP device {device}")
        _ctx[device] = h
    return _ctx[device]


def _check(st, ctx):
    if st != OK:
        raise LsgcpdError(st, load_library().lsgcpd_last_error(ctx).decode())


def _dev_tensor(a, shape_tail=None, name="array", device=None):
    torch = _torch()
    if not isinstance(a, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if not a.is_cuda:
        raise ValueError(f"{name} must be on a HIP device")
    if a.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not a.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and tuple(a.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape (n, {', '.join(map(str, shape_tail))})")
    if device is not None and a.device.index != device:
        raise ValueError(f"{name} is on another device")
    return a


def _ptr(a):
    return C.c_void_p(a.data_ptr()) if a is not None else C.c_void_p(0)


def _stream(device):
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _pose(R, t):
    p = Pose()
    R = np.asarray(R, dtype=np.float64).reshape(9)
    t = np.asarray(t, dtype=np.float64).reshape(3)
    for i in range(9):
        p.R[i] = R[i]
    for i in range(3):
        p.t[i] = t[i]
    return p


def _pose_np(p):
    return np.array(p.R[:], dtype=np.float64).reshape(3, 3), np.array(p.t[:], dtype=np.float64)


def normals(Y, k=10, alpha_max=30.0, lam=0.2, with_kappa=True):
    """Normals, surface variation and penalty alpha of every target point
    (lsgcpd_normals).  Returns (normals (M,3), kappa (M,) or None, alpha (M,))."""
    torch = _torch()
    Y = _dev_tensor(Y, (3,), "Y")
    dev = Y.device.index
    M = Y.shape[0]
    n = torch.empty((M, 3), dtype=torch.float32, device=Y.device)
    kap = torch.empty((M,), dtype=torch.float32, device=Y.device) if with_kappa else None
    al = torch.empty((M,), dtype=torch.float32, device=Y.device)
    ctx = context(dev)
    st = load_library().lsgcpd_normals(ctx, _ptr(Y), M, int(k), float(alpha_max), float(lam),
                                       _ptr(n), _ptr(kap), _ptr(al), _stream(dev))
    _check(st, ctx)
    return n, kap, al


@dataclass
class EStepResult:
    sigma2: float
    gamma: float
    V: float
    sumP: float
    outlier_mass: float
    nll: float
    pd: float
    stats: np.ndarray
    grad: np.ndarray
    hess: np.ndarray
    R_next: np.ndarray
    t_next: np.ndarray
    sigma2_next: float
    newton_iters: int
    gn_fallbacks: int
    P: object = None          # torch (M, N) float32 if requested
    colstats: object = None   # torch (N, 16) float64 if requested
    bf16_cross: bool = False  # the LSGCPD_BF16_CROSS path ran this E step


def estep(X, Y, nrm, alpha, R, t, sigma2, w0=0.1, V=0.0, pi=None, w=None, exact=False,
          backend="scalar", dump_P=False, colstats=False, noalloc=False, bf16=False):
    """One E step and the M step it implies (lsgcpd_estep; with noalloc,
    lsgcpd_estep_noalloc, which allocates no memory).  bf16: LSGCPD_BF16_CROSS
    (the matrix-core exponent where its error bound allows)."""
    torch = _torch()
    X = _dev_tensor(X, (3,), "X")
    dev = X.device.index
    Y = _dev_tensor(Y, (3,), "Y", dev)
    nrm = _dev_tensor(nrm, (3,), "normals", dev)
    alpha = _dev_tensor(alpha, None, "alpha", dev)
    N, M = X.shape[0], Y.shape[0]
    if nrm.shape[0] != M or alpha.numel() != M:
        raise ValueError("normals and alpha must have one row per target point")
    if pi is not None:
        pi = _dev_tensor(pi, None, "pi", dev)
        if pi.numel() != M:
            raise ValueError("pi must have M entries")
    if w is not None:
        w = _dev_tensor(w, None, "w", dev)
        if w.numel() != N:
            raise ValueError("w must have N entries")
    P = torch.empty((M, N), dtype=torch.float32, device=X.device) if dump_P else None
    cs = torch.empty((N, 16), dtype=torch.float64, device=X.device) if colstats else None
    flags = (EXACT_NORMALIZER if exact else 0) | _BACKENDS[backend] | (BF16_CROSS if bf16 else 0)
    out = EstepOut()
    pose = _pose(R, t)
    ctx = context(dev)
    lib = load_library()
    fn = lib.lsgcpd_estep_noalloc if noalloc else lib.lsgcpd_estep
    st = fn(ctx, _ptr(X), N, _ptr(Y), _ptr(nrm), _ptr(alpha), M, _ptr(pi), _ptr(w), float(w0),
            float(V), C.byref(pose), float(sigma2), flags, C.byref(out), _ptr(P), _ptr(cs),
            _stream(dev))
    _check(st, ctx)
    Rn, tn = _pose_np(out.pose_next)
    return EStepResult(sigma2=out.sigma2, gamma=out.gamma, V=out.V, sumP=out.sumP,
                       outlier_mass=out.outlier_mass, nll=out.nll, pd=out.pd,
                       stats=np.array(out.stats[:]), grad=np.array(out.grad[:]),
                       hess=np.array(out.hess[:]).reshape(6, 6), R_next=Rn, t_next=tn,
                       sigma2_next=out.sigma2_next, newton_iters=out.newton_iters,
                       gn_fallbacks=out.gn_fallbacks, P=P, colstats=cs,
                       bf16_cross=bool(out.bf16_cross))


@dataclass
class RegistrationResult:
    R: np.ndarray
    t: np.ndarray
    sigma2: float
    iters: int
    converged: bool
    gn_fallbacks: int
    nll: np.ndarray
    V: float
    w0: float = 0.0     # uniform outlier weight used
    n_used: int = 0     # points registered (after truncation)
    m_used: int = 0
    bf16_steps: int = 0  # E steps on the LSGCPD_BF16_CROSS path


def default_params():
    p = Params()
    load_library().lsgcpd_params_default(C.byref(p))
    return p


def _params(k, alpha_max, lam, w0, V, max_iter, tol, sigma2_init, newton_max, flags, eta):
    return Params(k=int(k), alpha_max=float(alpha_max), lambda_=float(lam), w0=float(w0),
                  V=float(V), max_iter=int(max_iter), tol=float(tol),
                  sigma2_init=float(sigma2_init), newton_max=int(newton_max), flags=flags,
                  eta=float(eta) if eta is not None else 0.0)


def _result(out, rep, nll):
    R, t = _pose_np(out)
    return RegistrationResult(R=R, t=t, sigma2=rep.sigma2, iters=rep.iters,
                              converged=bool(rep.converged), gn_fallbacks=rep.gn_fallbacks,
                              nll=nll, V=rep.V, w0=rep.w0, n_used=rep.n_used,
                              m_used=rep.m_used, bf16_steps=rep.bf16_steps)


def _init_pose(R0, t0):
    if R0 is None and t0 is None:
        return None
    return _pose(np.eye(3) if R0 is None else R0, np.zeros(3) if t0 is None else t0)


def register(X, Y, k=10, alpha_max=30.0, lam=0.2, w0=0.1, V=0.0, max_iter=50, tol=0.0,
             sigma2_init=0.0, newton_max=20, exact=False, backend="scalar", R0=None, t0=None,
             eta=None, graph=False, bf16=False):
    """Full LSG-CPD registration of X onto Y (lsgcpd_register).  eta: outlier
    ratio; w0 is then w_max (Sec. 3.2).  graph: replay the EM loop from a HIP
    graph recording (LSGCPD_GRAPH).  bf16: LSGCPD_BF16_CROSS."""
    X = _dev_tensor(X, (3,), "X")
    dev = X.device.index
    Y = _dev_tensor(Y, (3,), "Y", dev)
    p = _params(k, alpha_max, lam, w0, V, max_iter, tol, sigma2_init, newton_max,
                (EXACT_NORMALIZER if exact else 0) | _BACKENDS[backend] | (GRAPH if graph else 0)
                | (BF16_CROSS if bf16 else 0), eta)
    init = _init_pose(R0, t0)
    out = Pose()
    rep = Report()
    trace = (C.c_double * max(int(max_iter), 1))()
    ctx = context(dev)
    st = load_library().lsgcpd_register(ctx, _ptr(X), X.shape[0], _ptr(Y), Y.shape[0],
                                        C.byref(p), C.byref(init) if init is not None else None,
                                        C.byref(out), C.byref(rep), C.cast(trace, C.c_void_p),
                                        _stream(dev))
    _check(st, ctx)
    return _result(out, rep, np.array(trace[:rep.iters + rep.converged]))


def autotune(X, Y, k=10, alpha_max=30.0, lam=0.2, w0=0.1, V=0.0, max_iter=50, tol=0.0,
             sigma2_init=0.0, newton_max=20, exact=False, eta=None):
    """Measures the registration of X onto Y with several work-item counts
    and keeps the fastest for pairs of this size (lsgcpd_autotune); returns
    the count chosen."""
    X = _dev_tensor(X, (3,), "X")
    dev = X.device.index
    Y = _dev_tensor(Y, (3,), "Y", dev)
    p = _params(k, alpha_max, lam, w0, V, max_iter, tol, sigma2_init, newton_max,
                EXACT_NORMALIZER if exact else 0, eta)
    best = C.c_int32(0)
    ctx = context(dev)
    st = load_library().lsgcpd_autotune(ctx, _ptr(X), X.shape[0], _ptr(Y), Y.shape[0],
                                        C.byref(p), C.byref(best), _stream(dev))
    _check(st, ctx)
    return best.value


def depth_confidence(P, coef, e_min):
    """Confidence phi = e_min / e(z) of depth-sensor points, e(z) = coef[0] +
    coef[1] z + coef[2] z^2 (lsgcpd_depth_confidence); returns a float32 tensor."""
    torch = _torch()
    P = _dev_tensor(P, (3,), "P")
    dev = P.device.index
    phi = torch.empty((P.shape[0],), dtype=torch.float32, device=P.device)
    c = (C.c_double * 3)(*[float(v) for v in coef])
    ctx = context(dev)
    st = load_library().lsgcpd_depth_confidence(ctx, _ptr(P), P.shape[0], c, float(e_min),
                                                _ptr(phi), _stream(dev))
    _check(st, ctx)
    return phi


def register_cf(X, Y, phi_x=None, phi_y=None, threshold=0.0, k=10, alpha_max=30.0, lam=0.2,
                w0=0.1, V=0.0, max_iter=50, tol=0.0, sigma2_init=0.0, newton_max=20,
                exact=False, dense=False, R0=None, t0=None, eta=None, graph=False):
    """Registration with confidence filtering (lsgcpd_register_cf): priors
    from phi_y, outlier weights from phi_x, points below `threshold` dropped."""
    X = _dev_tensor(X, (3,), "X")
    dev = X.device.index
    Y = _dev_tensor(Y, (3,), "Y", dev)
    if phi_x is not None:
        phi_x = _dev_tensor(phi_x, None, "phi_x", dev)
        if phi_x.numel() != X.shape[0]:
            raise ValueError("phi_x must have N entries")
    if phi_y is not None:
        phi_y = _dev_tensor(phi_y, None, "phi_y", dev)
        if phi_y.numel() != Y.shape[0]:
            raise ValueError("phi_y must have M entries")
    p = _params(k, alpha_max, lam, w0, V, max_iter, tol, sigma2_init, newton_max,
                (EXACT_NORMALIZER if exact else 0) | (DENSE if dense else 0) |
                (GRAPH if graph else 0), eta)
    init = _init_pose(R0, t0)
    out = Pose()
    rep = Report()
    trace = (C.c_double * max(int(max_iter), 1))()
    ctx = context(dev)
    st = load_library().lsgcpd_register_cf(ctx, _ptr(X), _ptr(phi_x), X.shape[0], _ptr(Y),
                                           _ptr(phi_y), Y.shape[0], float(threshold), C.byref(p),
                                           C.byref(init) if init is not None else None,
                                           C.byref(out), C.byref(rep),
                                           C.cast(trace, C.c_void_p), _stream(dev))
    _check(st, ctx)
    return _result(out, rep, np.array(trace[:rep.iters + rep.converged]))


def register_batch(pairs, k=10, alpha_max=30.0, lam=0.2, w0=0.1, V=0.0, max_iter=50, tol=0.0,
                   sigma2_init=0.0, newton_max=20, exact=False, dense=False, init=None,
                   eta=None, graph=False, bf16=False):
    """Registers every (X, Y) of `pairs` in one batched pipeline
    (lsgcpd_register_batch); returns one RegistrationResult per pair (its
    `nll` holds the first and the last value of Eq. 4 only)."""
    n = len(pairs)
    if n < 1:
        raise ValueError("no pairs")
    Xs, Ys = [], []
    dev = None
    for X, Y in pairs:
        X = _dev_tensor(X, (3,), "X", dev)
        dev = X.device.index
        Xs.append(X)
        Ys.append(_dev_tensor(Y, (3,), "Y", dev))
    p = _params(k, alpha_max, lam, w0, V, max_iter, tol, sigma2_init, newton_max,
                (EXACT_NORMALIZER if exact else 0) | (DENSE if dense else 0) |
                (GRAPH if graph else 0) | (BF16_CROSS if bf16 else 0), eta)
    xp = (C.c_void_p * n)(*[_ptr(X) for X in Xs])
    yp = (C.c_void_p * n)(*[_ptr(Y) for Y in Ys])
    nn = (C.c_int64 * n)(*[X.shape[0] for X in Xs])
    mm = (C.c_int64 * n)(*[Y.shape[0] for Y in Ys])
    poses = None
    if init is not None:
        poses = (Pose * n)(*[_pose(R, t) for R, t in init])
    out = (Pose * n)()
    rep = (Report * n)()
    ctx = context(dev)
    st = load_library().lsgcpd_register_batch(ctx, n, C.cast(xp, C.c_void_p),
                                              C.cast(nn, C.c_void_p), C.cast(yp, C.c_void_p),
                                              C.cast(mm, C.c_void_p), C.byref(p), poses, out, rep,
                                              _stream(dev))
    _check(st, ctx)
    res = []
    for i in range(n):
        res.append(_result(out[i], rep[i], np.array([rep[i].nll_first, rep[i].nll_last])))
    return res


def profile_enable(on=True, device=0):
    """Turns event timing of the E-step kernels on or off (lsgcpd_profile_enable)."""
    ctx = context(device)
    _check(load_library().lsgcpd_profile_enable(ctx, 1 if on else 0), ctx)


def profile_read(reset=True, device=0):
    """Totals since the last reset: dict(launches, pairs, pair_kernel_ms, estep_ms,
    evaluated_pairs)."""
    ctx = context(device)
    p = Profile()
    _check(load_library().lsgcpd_profile_read(ctx, C.byref(p), 1 if reset else 0), ctx)
    return {"launches": p.launches, "pairs": p.pairs, "pair_kernel_ms": p.pair_kernel_ms,
            "estep_ms": p.estep_ms, "evaluated_pairs": p.evaluated_pairs}


def profile_launches(device=0):
    """Per-E-step times since the last reset, in launch order: two numpy
    arrays (pair kernel, whole E step) in microseconds
    (lsgcpd_profile_launches).  Read them before profile_read(reset=True)."""
    ctx = context(device)
    lib = load_library()
    n = C.c_int64(0)
    _check(lib.lsgcpd_profile_launches(ctx, None, None, 0, C.byref(n)), ctx)
    a = (C.c_double * max(n.value, 1))()
    b = (C.c_double * max(n.value, 1))()
    _check(lib.lsgcpd_profile_launches(ctx, a, b, n.value, C.byref(n)), ctx)
    return np.array(a[:n.value]), np.array(b[:n.value])


PROPOSAL_PARAMS = 108425
PROPOSAL_NORM = 25


def proposal_inputs(pairs, P, Q=None):
    """Encoder inputs of the (X, Y) pairs (lsgcpd_proposal_inputs): Xn, Yn
    (npairs, P, 3) float32 and norm (npairs, 25: mu_X, mu_Y, s, F_X, F_Y)
    float64 device tensors.  Q: optional (npairs, 3, 3) rotations of the
    sources."""
    torch = _torch()
    n = len(pairs)
    if n < 1:
        raise ValueError("no pairs")
    Xs, Ys, dev = [], [], None
    for X, Y in pairs:
        X = _dev_tensor(X, (3,), "X", dev)
        dev = X.device.index
        Xs.append(X)
        Ys.append(_dev_tensor(Y, (3,), "Y", dev))
    device = Xs[0].device
    Xn = torch.empty((n, P, 3), dtype=torch.float32, device=device)
    Yn = torch.empty((n, P, 3), dtype=torch.float32, device=device)
    norm = torch.empty((n, PROPOSAL_NORM), dtype=torch.float64, device=device)
    Qh = None
    if Q is not None:
        Qh = np.ascontiguousarray(Q, dtype=np.float64).reshape(n, 9)
    xp = (C.c_void_p * n)(*[_ptr(X) for X in Xs])
    yp = (C.c_void_p * n)(*[_ptr(Y) for Y in Ys])
    nn = (C.c_int64 * n)(*[X.shape[0] for X in Xs])
    mm = (C.c_int64 * n)(*[Y.shape[0] for Y in Ys])
    ctx = context(dev)
    st = load_library().lsgcpd_proposal_inputs(ctx, n, C.cast(xp, C.c_void_p), C.cast(nn, C.c_void_p),
                                               C.cast(yp, C.c_void_p), C.cast(mm, C.c_void_p),
                                               _host(Qh), int(P), _ptr(Xn), _ptr(Yn), _ptr(norm),
                                               _stream(dev))
    _check(st, ctx)
    return Xn, Yn, norm


def _f32(a, n, name, dev):
    a = _dev_tensor(a, None, name, dev)
    if a.numel() != n:
        raise ValueError(f"{name} must have {n} entries")
    return a


def proposal_forward(theta, Xn, Yn, norm):
    """Predicted poses (lsgcpd_proposal_forward): a (npairs, 12) float64
    device tensor, R row-major then t, world units."""
    torch = _torch()
    if Xn.dim() != 3 or Xn.shape[2] != 3 or Yn.shape != Xn.shape:
        raise ValueError("Xn and Yn must have shape (npairs, P, 3)")
    n, P = Xn.shape[0], Xn.shape[1]
    dev = Xn.device.index
    theta = _f32(theta, PROPOSAL_PARAMS, "theta", dev)
    pose = torch.empty((n, 12), dtype=torch.float64, device=Xn.device)
    ctx = context(dev)
    st = load_library().lsgcpd_proposal_forward(ctx, _ptr(theta), n, P, _ptr(Xn), _ptr(Yn),
                                                _ptr(norm), _ptr(pose), _stream(dev))
    _check(st, ctx)
    return pose


def _host(a):
    return C.c_void_p(a.ctypes.data) if a is not None else C.c_void_p(0)


def proposal_train_step(theta, m, v, step, lr, Xn, Yn, norm, label, index=None,
                        want_argmax=False, want_grad=False):
    """One Adam step of the proposal on a batch (lsgcpd_proposal_train_step);
    theta, m, v (float32 device tensors of PROPOSAL_PARAMS) are updated in
    place.  Xn, Yn, norm: stored inputs (proposal_inputs); label (B, 12) and
    index (B,): host arrays.  Returns the device tensors (loss per pair,
    argmax or None, gradient or None)."""
    torch = _torch()
    dev = Xn.device.index
    label = np.ascontiguousarray(label, np.float64).reshape(-1, 12)
    B = label.shape[0]
    P = Xn.shape[1]
    for name, a in (("theta", theta), ("m", m), ("v", v)):
        if a.dtype != torch.float32 or a.numel() != PROPOSAL_PARAMS or not a.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 tensor of {PROPOSAL_PARAMS}")
    idx = None if index is None else np.ascontiguousarray(index, np.int32).reshape(B)
    loss = torch.empty(B, dtype=torch.float64, device=Xn.device)
    am = torch.empty((B, 2, 256), dtype=torch.int32, device=Xn.device) if want_argmax else None
    g = torch.empty(PROPOSAL_PARAMS, dtype=torch.float32, device=Xn.device) if want_grad else None
    ctx = context(dev)
    st = load_library().lsgcpd_proposal_train_step(
        ctx, _ptr(theta), _ptr(m), _ptr(v), int(step), float(lr), B, P, _ptr(Xn), _ptr(Yn),
        _ptr(norm), int(Xn.shape[0]), _host(idx), _host(label), _ptr(loss), _ptr(am), _ptr(g),
        _stream(dev))
    _check(st, ctx)
    return loss, am, g


def register_proposed(pairs, theta, P=512, accept=0.1, k=10, alpha_max=30.0, lam=0.2, w0=0.1,
                      V=0.0, max_iter=50, tol=0.0, sigma2_init=0.0, newton_max=20, exact=False,
                      eta=None):
    """Registers every (X, Y) of `pairs` from the learned proposal's pose,
    with 24-start EM for the pairs it does not accept
    (lsgcpd_register_proposed).  Returns (results, fallback flags)."""
    n = len(pairs)
    if n < 1:
        raise ValueError("no pairs")
    Xs, Ys, dev = [], [], None
    for X, Y in pairs:
        X = _dev_tensor(X, (3,), "X", dev)
        dev = X.device.index
        Xs.append(X)
        Ys.append(_dev_tensor(Y, (3,), "Y", dev))
    theta = _dev_tensor(theta, None, "theta", dev)
    if theta.numel() != PROPOSAL_PARAMS:
        raise ValueError(f"theta must have {PROPOSAL_PARAMS} entries")
    p = _params(k, alpha_max, lam, w0, V, max_iter, tol, sigma2_init, newton_max,
                EXACT_NORMALIZER if exact else 0, eta)
    xp = (C.c_void_p * n)(*[_ptr(X) for X in Xs])
    yp = (C.c_void_p * n)(*[_ptr(Y) for Y in Ys])
    nn = (C.c_int64 * n)(*[X.shape[0] for X in Xs])
    mm = (C.c_int64 * n)(*[Y.shape[0] for Y in Ys])
    out = (Pose * n)()
    rep = (Report * n)()
    fb = (C.c_int32 * n)()
    ctx = context(dev)
    st = load_library().lsgcpd_register_proposed(ctx, n, C.cast(xp, C.c_void_p),
                                                 C.cast(nn, C.c_void_p), C.cast(yp, C.c_void_p),
                                                 C.cast(mm, C.c_void_p), C.byref(p), _ptr(theta),
                                                 int(P), float(accept), out, rep,
                                                 C.cast(fb, C.c_void_p), _stream(dev))
    _check(st, ctx)
    res = [_result(out[i], rep[i], np.array([rep[i].nll_first, rep[i].nll_last]))
           for i in range(n)]
    return res, np.array(fb[:], dtype=np.int32)
