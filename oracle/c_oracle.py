"""ctypes wrapper of estep_ref.c, the plain FP64 C form of the oracle's E step
(test infrastructure only).  Build with oracle.c_oracle.build()."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from . import lsgcpd_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "estep_ref.c")
LIB = os.path.join(HERE, "liboracle_ref.so")
_lib = None


def build():
    """gcc -O2, OpenMP, no floating-point contraction (always recompiles)."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", SRC,
                    "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        vp, i64, d = C.c_void_p, C.c_int64, C.c_double
        L.oracle_estep_columns.restype = None
        L.oracle_estep_columns.argtypes = [vp, i64, vp, vp, vp, i64, vp, vp, d, d, vp, vp, d,
                                           C.c_int, vp, i64, vp]
        L.oracle_pair_sqdist_sum.restype = d
        L.oracle_pair_sqdist_sum.argtypes = [vp, i64, vp, i64, vp, vp]
        L.oracle_knn.restype = None
        L.oracle_knn.argtypes = [vp, i64, C.c_int, vp, i64, vp]
        L.oracle_threads.restype = C.c_int
        L.oracle_set_threads.restype = None
        L.oracle_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def threads():
    return lib().oracle_threads()


def set_threads(n):
    """OpenMP threads of the later calls (for timing runs)."""
    lib().oracle_set_threads(int(n))


def estep_columns(X, Y, normals, alpha, R, t, sigma2, w0=0.1, V=None, pi=None, w=None,
                  exact_normalizer=False, sources=None):
    """Per-source sums of the posterior (see estep_ref.c) -> (Columns, Ksum)
    for the given sources (all by default).  float32 clouds, normals, alpha."""
    X = np.ascontiguousarray(X, np.float32)
    Y = np.ascontiguousarray(Y, np.float32)
    nrm = np.ascontiguousarray(normals, np.float32)
    al = np.ascontiguousarray(alpha, np.float32)
    if V is None:
        V = O.working_volume(Y)
    R = np.ascontiguousarray(R, np.float64)
    t = np.ascontiguousarray(t, np.float64)
    pi = None if pi is None else np.ascontiguousarray(pi, np.float64)
    w = None if w is None else np.ascontiguousarray(w, np.float64)
    src = None if sources is None else np.ascontiguousarray(sources, np.int64)
    S = len(X) if src is None else len(src)
    out = np.zeros((S, 16))
    lib().oracle_estep_columns(_p(X), len(X), _p(Y), _p(nrm), _p(al), len(Y), _p(pi), _p(w),
                               float(w0), float(V), _p(R), _p(t), float(sigma2),
                               1 if exact_normalizer else 0, _p(src), S, _p(out))
    cols = O.Columns(p=out[:, 1], A=out[:, 2:11].reshape(-1, 3, 3), B=out[:, 11:14],
                     C=out[:, 14], b=None, c=out[:, 15])
    return cols, out[:, 0]


def register_columns_fn(X, Y, normals, alpha, w0, V, exact_normalizer=False, pi=None, w=None):
    """An `estep_columns` callback for lsgcpd_oracle.register: the C E step
    plus the negative log-likelihood of Eq. (4).  pi / w: per-point priors and
    outlier weights (None: 1/M and w0)."""
    logw = np.log(w0) if w is None else np.log(np.asarray(w, np.float64))

    def fn(R, t, s2):
        cols, ksum = estep_columns(X, Y, normals, alpha, R, t, s2, w0=w0, V=V, pi=pi, w=w,
                                   exact_normalizer=exact_normalizer)
        gamma = (2.0 * np.pi * s2) ** 1.5 / V
        nll = -float(np.sum(logw + np.log(ksum + gamma) - 1.5 * np.log(2 * np.pi * s2)))
        return cols, nll
    return fn


def knn_indices(Y, k, queries=None):
    Y = np.ascontiguousarray(Y, np.float32)
    q = None if queries is None else np.ascontiguousarray(queries, np.int64)
    Q = len(Y) if q is None else len(q)
    out = np.zeros((Q, k), np.int64)
    lib().oracle_knn(_p(Y), len(Y), int(k), _p(q), Q, _p(out))
    return out


def sigma2_init(X, Y, R, t):
    X = np.ascontiguousarray(X, np.float32)
    Y = np.ascontiguousarray(Y, np.float32)
    tot = lib().oracle_pair_sqdist_sum(_p(X), len(X), _p(Y), len(Y),
                                       _p(np.ascontiguousarray(R, np.float64)),
                                       _p(np.ascontiguousarray(t, np.float64)))
    return tot / (3.0 * len(X) * len(Y))
