"""Pins for the oracle's M step (Sec. 3.5, Eq. 11-13) and the EM loop."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

import datagen
from oracle import lsgcpd_oracle as O


def _problem(seed, M=12, N=10, alpha_hi=15.0):
    rng = np.random.default_rng(seed)
    Y = rng.normal(size=(M, 3)) * 0.5
    X = Y[:N] @ datagen.random_rotation(rng, 0.2).T + rng.normal(size=(N, 3)) * 0.05
    nrm = rng.normal(size=(M, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    alpha = rng.uniform(0, alpha_hi, size=M)
    R = datagen.random_rotation(rng, 0.1)
    t = rng.normal(size=3) * 0.05
    return rng, X, Y, nrm, alpha, R, t


def _F(P, X, Y, nrm, alpha, g, s2):
    """sum_mn P_mn (g x~ - y~)^T Sigma~^{-1} (g x~ - y~), the quantity whose
    right derivatives Eq. (11)-(12) print."""
    d = O.mahalanobis_sq(X @ g[:3, :3].T + g[:3, 3], Y, nrm, alpha)
    return float(np.sum(P * d)) / s2


def test_se3_exp_matches_expm():
    rng = np.random.default_rng(0)
    for scale in (1e-9, 1e-4, 0.3, 2.5):
        xi = rng.normal(size=6) * scale
        np.testing.assert_allclose(O.se3_exp(xi), scipy.linalg.expm(O.se3_hat(xi)),
                                   rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1])
def test_grad_hess_finite_differences(seed):
    rng, X, Y, nrm, alpha, R, t = _problem(seed)
    s2 = 0.04
    es = O.estep(X, Y, nrm, alpha, R, t, s2, w0=0.1, V=2.0)
    g = O.homog(R, t)
    grad, H = O.grad_hess_literal(es.P, X, Y, nrm, alpha, R, t, s2)
    h = 1e-5
    E6 = np.eye(6)
    f = lambda xi: _F(es.P, X, Y, nrm, alpha, g @ O.se3_exp(xi), s2)
    fd = np.array([(f(h * E6[i]) - f(-h * E6[i])) / (2 * h) for i in range(6)])
    np.testing.assert_allclose(grad, fd, rtol=1e-7, atol=1e-7 * np.abs(fd).max())
    Hs = 0.5 * (H + H.T)
    f0 = f(np.zeros(6))
    Hfd = np.empty((6, 6))
    for i in range(6):
        for j in range(6):
            Hfd[i, j] = (f(h * (E6[i] + E6[j])) - f(h * (E6[i] - E6[j]))
                         - f(h * (E6[j] - E6[i])) + f(-h * (E6[i] + E6[j]))) / (4 * h * h)
    np.testing.assert_allclose(Hs, Hfd, rtol=1e-4, atol=1e-4 * np.abs(Hfd).max())
    # the per-source form equals the printed double sums
    cols = O.columns(es.P, X, Y, nrm, alpha, R, t)
    g2, H2 = O.grad_hess(cols, X, R, t, s2)
    np.testing.assert_allclose(g2, grad, rtol=1e-10, atol=1e-12 * np.abs(grad).max())
    np.testing.assert_allclose(H2, H, rtol=1e-10, atol=1e-12 * np.abs(H).max())


def _procrustes(P, X, Y):
    """Weighted Procrustes: argmin_{R,t} sum P_mn |R x_n + t - y_m|^2, the
    closed-form rigid M step of CPD (Myronenko & Song, Fig. 2)."""
    Np = P.sum()
    mx = X.T @ P.sum(axis=0) / Np
    my = Y.T @ P.sum(axis=1) / Np
    A = (Y - my).T @ P @ (X - mx)
    U, _, Vt = np.linalg.svd(A)
    Dg = np.diag([1.0, 1.0, np.linalg.det(U @ Vt)])
    R = U @ Dg @ Vt
    return R, my - R @ mx


@pytest.mark.parametrize("seed", [2, 3, 4])
def test_isotropic_mstep_is_weighted_procrustes(seed):
    rng, X, Y, nrm, alpha, R, t = _problem(seed, M=30, N=25)
    a0 = np.zeros(len(Y))
    s2 = 0.05
    es = O.estep(X, Y, nrm, a0, R, t, s2, w0=0.1, V=2.0)
    cols = O.columns(es.P, X, Y, nrm, a0, R, t)
    ms = O.mstep(cols, X, R, t, s2)
    Rp, tp = _procrustes(es.P, X, Y)
    assert O.rotation_error_deg(ms.R, Rp) < 1e-9
    np.testing.assert_allclose(ms.t, tp, atol=1e-11)
    # CPD's variance update: sum P |R x + t - y|^2 / (3 N_P)
    d = np.sum(((X @ Rp.T + tp)[None] - Y[:, None]) ** 2, axis=2)
    assert ms.sigma2 == pytest.approx(np.sum(es.P * d) / (3 * es.P.sum()), rel=1e-10)


@pytest.mark.parametrize("seed", [5, 6])
def test_mstep_matches_bfgs_and_is_stationary(seed):
    rng, X, Y, nrm, alpha, R, t = _problem(seed, M=20, N=15, alpha_hi=40.0)
    s2 = 0.03
    es = O.estep(X, Y, nrm, alpha, R, t, s2, w0=0.1, V=2.0)
    cols = O.columns(es.P, X, Y, nrm, alpha, R, t)
    ms = O.mstep(cols, X, R, t, s2)
    g = O.homog(R, t)
    f = lambda xi: _F(es.P, X, Y, nrm, alpha, g @ O.se3_exp(xi), 1.0)
    res = scipy.optimize.minimize(f, np.zeros(6), method="BFGS",
                                  options={"gtol": 1e-13, "maxiter": 2000})
    gb = g @ O.se3_exp(res.x)
    # BFGS with finite-difference gradients is accurate to about 1e-8
    assert O.rotation_error_deg(ms.R, gb[:3, :3]) < 2e-5
    np.testing.assert_allclose(ms.t, gb[:3, 3], atol=1e-7)
    grad, _ = O.grad_hess_literal(es.P, X, Y, nrm, alpha, ms.R, ms.t, s2)
    gscale, _ = O.grad_hess_literal(es.P, X, Y, nrm, alpha, R, t, s2)
    assert np.max(np.abs(grad)) <= 1e-9 * max(1.0, np.max(np.abs(gscale)))
    # sigma^2: stationary point of Q in sigma^2 at the new pose
    d = O.mahalanobis_sq(X @ ms.R.T + ms.t, Y, nrm, alpha)
    assert ms.sigma2 == pytest.approx(np.sum(es.P * d) / (3 * es.P.sum()), rel=1e-10)


def _small_pair(trial, M=300, N=300, angle=30.0):
    return datagen.range_scanner_pair(trial=trial, M=M, N=N, angle_deg=angle)


def test_em_nll_monotone():
    p = _small_pair(0)
    reg = O.register(p.X, p.Y, k=10, max_iter=30)
    nll = np.array(reg.nll)
    assert np.all(np.diff(nll) <= 1e-9 * np.abs(nll[1:]))
    assert O.rotation_error_deg(reg.R, p.R_gt) < 2.0


def test_em_exact_recovery_noise_free():
    rng = np.random.default_rng(21)
    Y = datagen._sample_box_sphere(rng, 400)
    Rg = datagen.random_rotation(rng, math.radians(25.0))
    tg = rng.uniform(-0.1, 0.1, size=3)
    X = (Y - tg) @ Rg          # g*(x) = Rg x + tg maps X exactly onto Y
    reg = O.register(X, Y, k=10, max_iter=100)
    diag = O.bbox_diag(Y)
    assert O.rotation_error_deg(reg.R, Rg) < 1e-4
    assert O.translation_error(reg.t, tg) < 1e-6 * diag


def test_em_source_motion_composes():
    p = _small_pair(1, M=250, N=250)
    rng = np.random.default_rng(3)
    Rh = datagen.random_rotation(rng, 0.15)
    th = rng.normal(size=3) * 0.05
    X = p.X.astype(np.float64)
    a = O.register(X, p.Y, max_iter=25)
    b = O.register(X @ Rh.T + th, p.Y, max_iter=25, R0=Rh.T, t0=-(Rh.T @ th))
    # starting b at h^{-1} reproduces a's iterates: the result is g h^{-1}
    assert O.rotation_error_deg(b.R @ Rh, a.R) < 1e-7
    np.testing.assert_allclose(b.R @ Rh, a.R, atol=1e-8)
    np.testing.assert_allclose(b.t - (a.t - a.R @ Rh.T @ th), 0, atol=1e-8)


def test_em_alpha_zero_is_rigid_cpd():
    """alpha_max = 0 with V = N: every iteration equals rigid CPD (posterior
    of CPD with w, Procrustes, CPD's sigma^2 update)."""
    p = _small_pair(2, M=200, N=180)
    X, Y = p.X.astype(np.float64), p.Y.astype(np.float64)
    N, M = len(X), len(Y)
    w, iters = 0.1, 15
    reg = O.register(X, Y, alpha_max=0.0, w0=w, V=float(N), max_iter=iters)
    R, t = np.eye(3), np.zeros(3)
    s2 = np.sum((X[None] - Y[:, None]) ** 2) / (3 * M * N)
    for _ in range(iters):
        Xg = X @ R.T + t
        E = np.exp(-np.sum((Xg[None] - Y[:, None]) ** 2, axis=2) / (2 * s2))
        c = (2 * math.pi * s2) ** 1.5 * w / (1 - w) * M / N
        P = E / (E.sum(axis=0) + c)
        R, t = _procrustes(P, X, Y)
        d = np.sum(((X @ R.T + t)[None] - Y[:, None]) ** 2, axis=2)
        s2 = np.sum(P * d) / (3 * P.sum())
    assert O.rotation_error_deg(reg.R, R) < 1e-8
    np.testing.assert_allclose(reg.t, t, atol=1e-10)
    assert reg.sigma2 == pytest.approx(s2, rel=1e-8)
