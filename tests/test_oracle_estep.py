"""Pins for the oracle's E step (Eq. 1, 2, 4, 5, 9, 10) and the per-source
aggregates."""
import math

import numpy as np
import pytest
from scipy.stats import multivariate_normal

import datagen
from oracle import lsgcpd_oracle as O


def _case(seed, M=9, N=7, spread=0.4):
    rng = np.random.default_rng(seed)
    Y = rng.normal(size=(M, 3)) * spread
    X = rng.normal(size=(N, 3)) * spread
    nrm = datagen.random_unit_normals(rng, M).astype(np.float64)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)   # unit in float64
    alpha = rng.uniform(0, 20, size=M)
    R = datagen.random_rotation(rng, 0.3)
    t = rng.normal(size=3) * 0.1
    return rng, X, Y, nrm, alpha, R, t


def _mixture_direct(X, Y, nrm, alpha, R, t, s2, w, pi, V, exact):
    """Eq. (1), (2), (5) with scipy's Gaussian density.  Component covariance
    Sigma_m = sigma^2 (alpha n n^T + I)^{-1}.  With the printed normaliser the
    density is divided by sqrt(1 + alpha_m) (det Sigma_m^{-1/2} dropped)."""
    M, N = len(Y), len(X)
    Xg = X @ R.T + t
    pdf = np.zeros((M, N))
    for m in range(M):
        Sinv = (alpha[m] * np.outer(nrm[m], nrm[m]) + np.eye(3)) / s2
        pdf[m] = multivariate_normal(mean=Y[m], cov=np.linalg.inv(Sinv)).pdf(Xg)
        if not exact:
            pdf[m] /= math.sqrt(1.0 + alpha[m])
    num = (1 - w)[None, :] * pi[:, None] * pdf
    dens = w / V + num.sum(axis=0)
    return num / dens[None, :], dens


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_posterior_equals_gaussian_mixture(seed, exact):
    rng, X, Y, nrm, alpha, R, t = _case(seed)
    w = rng.uniform(0.05, 0.6, size=len(X))
    pi = rng.uniform(0.5, 1.5, size=len(Y))
    pi /= pi.sum()
    s2, V = 0.05, 3.0
    es = O.estep(X, Y, nrm, alpha, R, t, s2, V=V, pi=pi, w=w, exact_normalizer=exact)
    P, dens = _mixture_direct(X, Y, nrm, alpha, R, t, s2, w, pi, V, exact)
    np.testing.assert_allclose(es.P, P, rtol=1e-12, atol=1e-300)
    assert es.nll == pytest.approx(-np.sum(np.log(dens)), rel=1e-12)
    # columns: components plus the outlier posterior w_n p_o / p(x_n) sum to 1
    np.testing.assert_allclose(es.P.sum(axis=0) + (w / V) / dens, 1.0, rtol=1e-13)


def test_posterior_equals_matrix_recast():
    """Eq. (10): K = C o exp(-(D A + B) / (2 sigma^2)) with
    A = (N R X^T + N t 1^T - s 1^T)^(o2),
    B = Q + |t|^2 1 1^T + 2 (1 t^T R X^T - Y R X^T - Y t 1^T),
    Q_mn = |x_n|^2 + |y_m|^2 (the printed 't^T t I' read as |t|^2 everywhere)."""
    rng, X, Y, nrm, alpha, R, t = _case(5, M=11, N=13)
    w0, s2, V = 0.2, 0.08, 2.0
    es = O.estep(X, Y, nrm, alpha, R, t, s2, w0=w0, V=V)
    M, N = len(Y), len(X)
    one_m, one_n = np.ones((M, 1)), np.ones((N, 1))
    s = np.sum(Y * nrm, axis=1)[:, None]
    A = (nrm @ R @ X.T + nrm @ t[:, None] @ one_n.T - s @ one_n.T) ** 2
    Q = np.sum(X * X, axis=1)[None, :] + np.sum(Y * Y, axis=1)[:, None]
    B = Q + (t @ t) * one_m @ one_n.T + 2 * (one_m @ t[None, :] @ R @ X.T
                                              - Y @ R @ X.T - Y @ t[:, None] @ one_n.T)
    C = np.full((M, N), (1 - w0) / w0 / M)
    K = C * np.exp(-(np.diag(alpha) @ A + B) / (2 * s2))
    gamma = (2 * math.pi * s2) ** 1.5 / V
    np.testing.assert_allclose(es.P, K / (K.sum(axis=0) + gamma), rtol=1e-11)
    assert es.gamma == pytest.approx(gamma, rel=1e-15)


def test_alpha_zero_is_rigid_cpd_posterior():
    """alpha = 0 and V = N (p_o = 1/N): the posterior of rigid CPD (Myronenko &
    Song), P = exp(-|x - y_m|^2/2s2) / (sum_k exp(.) + (2 pi s2)^{3/2} w/(1-w) M/N)."""
    rng, X, Y, nrm, alpha, R, t = _case(7, M=15, N=12)
    w, s2 = 0.3, 0.1
    M, N = len(Y), len(X)
    es = O.estep(X, Y, nrm, np.zeros(M), R, t, s2, w0=w, V=float(N))
    Xg = X @ R.T + t
    E = np.exp(-np.sum((Xg[None] - Y[:, None]) ** 2, axis=2) / (2 * s2))
    c = (2 * math.pi * s2) ** 1.5 * w / (1 - w) * M / N
    np.testing.assert_allclose(es.P, E / (E.sum(axis=0) + c), rtol=1e-13)


def test_equivariance_and_invariance():
    rng, X, Y, nrm, alpha, R, t = _case(9, M=10, N=8)
    es = O.estep(X, Y, nrm, alpha, R, t, 0.07, w0=0.1, V=2.0)
    pm, pn = rng.permutation(10), rng.permutation(8)
    es2 = O.estep(X[pn], Y[pm], nrm[pm], alpha[pm], R, t, 0.07, w0=0.1, V=2.0)
    np.testing.assert_allclose(es2.P, es.P[np.ix_(pm, pn)], rtol=1e-13)
    # move the target and its normals rigidly by h, compose h into g
    Rh = datagen.random_rotation(rng, 1.1)
    th = rng.normal(size=3)
    es3 = O.estep(X, Y @ Rh.T + th, nrm @ Rh.T, alpha, Rh @ R, Rh @ t + th, 0.07, w0=0.1, V=2.0)
    np.testing.assert_allclose(es3.P, es.P, rtol=1e-11)
    # normal sign is irrelevant
    es4 = O.estep(X, Y, -nrm, alpha, R, t, 0.07, w0=0.1, V=2.0)
    np.testing.assert_allclose(es4.P, es.P, rtol=1e-14)


def test_limits():
    rng, X, Y, nrm, alpha, R, t = _case(11)
    big = O.estep(X, Y, nrm, alpha, R, t, 0.05, w0=0.1, V=1e300)
    np.testing.assert_allclose(big.P.sum(axis=0), 1.0, rtol=1e-14)   # softmax
    wide = O.estep(X, Y, nrm, alpha, R, t, 1e8, w0=0.1, V=1.0)
    assert np.all(wide.P < 1e-10)                                       # all outliers
    # equal distances over m: the column is uniform
    Yc = np.zeros((6, 3))
    eq = O.estep(X, Yc, np.tile([0, 0, 1.0], (6, 1)), np.full(6, 3.0), R, t, 0.2, w0=0.1, V=2.0)
    np.testing.assert_allclose(eq.P, eq.P[:1].repeat(6, axis=0), rtol=1e-15)


def test_columns_definitions():
    rng, X, Y, nrm, alpha, R, t = _case(13, M=8, N=6)
    es = O.estep(X, Y, nrm, alpha, R, t, 0.07, w0=0.1, V=2.0)
    cols = O.columns(es.P, X, Y, nrm, alpha, R, t)
    Xg = X @ R.T + t
    for n in range(len(X)):
        A = sum(es.P[m, n] * (np.eye(3) + alpha[m] * np.outer(nrm[m], nrm[m])) for m in range(len(Y)))
        Bv = sum(es.P[m, n] * (np.eye(3) + alpha[m] * np.outer(nrm[m], nrm[m])) @ Y[m] for m in range(len(Y)))
        c = sum(es.P[m, n] * ((Xg[n] - Y[m]) @ (Xg[n] - Y[m]) + alpha[m] * (nrm[m] @ (Xg[n] - Y[m])) ** 2)
                for m in range(len(Y)))
        np.testing.assert_allclose(cols.A[n], A, rtol=1e-13)
        np.testing.assert_allclose(cols.B[n], Bv, rtol=1e-13)
        assert cols.c[n] == pytest.approx(c, rel=1e-12)
        assert cols.p[n] == pytest.approx(es.P[:, n].sum(), rel=1e-14)
    # sum P d at any pose from the aggregates equals the dense double sum
    R2 = datagen.random_rotation(rng, 0.5)
    t2 = rng.normal(size=3)
    d2 = O.mahalanobis_sq(X @ R2.T + t2, Y, nrm, alpha)
    assert O.pd_of(cols, X, R2, t2) == pytest.approx(np.sum(es.P * d2), rel=1e-12)
    assert O.pd_of(cols, X, R, t) == pytest.approx(np.sum(cols.c), rel=1e-12)
