"""Pins for the oracle's outlier weight from the outlier ratio (Sec. 3.2) and
its confidence filtering (Sec. 3.3): the defining property of w_max (expected
outlier count eta N when every density sits at its bound), the peak density
of a Gaussian from scipy, a closed form of the posterior that w0 = w_max
implies, hand-computed confidences, brute-force truncation, and the uniform
special case."""
import math

import numpy as np
import pytest
from scipy.stats import multivariate_normal

import datagen
from oracle import lsgcpd_oracle as O


def _targets(seed, M=11):
    rng = np.random.default_rng(seed)
    Y = rng.normal(size=(M, 3)) * 0.3
    nrm = rng.normal(size=(M, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    alpha = rng.uniform(0.0, 25.0, size=M)
    pi = rng.dirichlet(np.ones(M))
    return rng, Y, nrm, alpha, pi


@pytest.mark.parametrize("exact", [False, True])
def test_component_peak_is_the_density_at_its_mean(exact):
    _, Y, nrm, alpha, _ = _targets(0)
    s2 = 0.013
    c = O.component_peak(alpha, s2, exact)
    for m in range(len(Y)):
        Sinv = (alpha[m] * np.outer(nrm[m], nrm[m]) + np.eye(3)) / s2
        peak = multivariate_normal(mean=Y[m], cov=np.linalg.inv(Sinv)).pdf(Y[m])
        if not exact:  # the printed E step drops det(Sigma_m^-1)^{1/2} / sigma^-3
            peak /= math.sqrt(1.0 + alpha[m])
        assert c[m] == pytest.approx(peak, rel=1e-12)


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("eta", [0.05, 0.3, 0.8])
def test_wmax_gives_eta_outliers_when_densities_reach_their_bound(eta, exact):
    # Sec. 3.2: with p(g(x_n)|m) = c_m for every m, the outlier posterior of
    # every point equals eta exactly when w0 = w_max.  All targets at one
    # point and every source on it make d_mn = 0, so the oracle's own E step
    # evaluates that situation.
    rng, _, nrm, alpha, pi = _targets(1)
    y0 = np.array([0.2, -0.1, 0.4])
    Y = np.tile(y0, (len(alpha), 1))
    X = np.tile(y0, (5, 1))
    s2, V = 0.02, 0.7
    w0 = O.outlier_weight_max(eta, V, pi, alpha, s2, exact)
    es = O.estep(X, Y, nrm, alpha, np.eye(3), np.zeros(3), s2, w0=w0, V=V, pi=pi,
                 exact_normalizer=exact)
    outlier = 1.0 - es.P.sum(axis=0)
    np.testing.assert_allclose(outlier, eta, rtol=1e-12)
    # the same from the expression of the outlier posterior with c_m from scipy
    c = np.array([multivariate_normal(mean=y0, cov=np.linalg.inv(
        (a * np.outer(n, n) + np.eye(3)) / s2)).pdf(y0) / (1.0 if exact else math.sqrt(1 + a))
        for a, n in zip(alpha, nrm)])
    r = w0 / (1.0 - w0) / V
    assert r / (r + np.sum(pi * c)) == pytest.approx(eta, rel=1e-12)


def test_wmax_limits_and_monotonicity():
    _, _, _, alpha, pi = _targets(2)
    assert O.outlier_weight_max(0.0, 1.0, pi, alpha, 0.1) == 0.0
    ws = [O.outlier_weight_max(e, 2.0, pi, alpha, 0.1) for e in np.linspace(0.01, 0.99, 30)]
    assert all(0.0 < w < 1.0 for w in ws)
    assert all(b > a for a, b in zip(ws, ws[1:]))
    # V S = 1 and eta = 1/2: w_max = (1/2) / (1/2 + 1/2)
    s2 = 1.0 / (2.0 * math.pi)       # c_m = 1 with the printed normaliser
    assert O.outlier_weight_max(0.5, 1.0, None, alpha, s2) == pytest.approx(0.5, rel=1e-15)
    with pytest.raises(ValueError):
        O.outlier_weight_max(1.0, 1.0, pi, alpha, 0.1)


@pytest.mark.parametrize("exact", [False, True])
def test_wmax_posterior_depends_on_sigma2_only_through_the_exponent(exact):
    # With w0 = w_max(sigma^2): rho gamma^-1 ... cancels to
    # P_mn = pi_m e_mn / (sum_m pi_m e_mn + eta / (1 - eta) sum_m pi_m chat_m)
    # with e_mn the (normalised) exponential and chat_m = c_m (2 pi s2)^{3/2}.
    rng, Y, nrm, alpha, pi = _targets(3)
    X = rng.normal(size=(8, 3)) * 0.3
    R, t = datagen.random_rotation(rng, 0.2), rng.normal(size=3) * 0.05
    eta, V = 0.25, 1.7
    for s2 in (0.004, 0.05, 0.6):
        w0 = O.outlier_weight_max(eta, V, pi, alpha, s2, exact)
        es = O.estep(X, Y, nrm, alpha, R, t, s2, w0=w0, V=V, pi=pi, exact_normalizer=exact)
        d = O.mahalanobis_sq(X @ R.T + t, Y, nrm, alpha)
        chat = np.sqrt(1.0 + alpha) if exact else np.ones_like(alpha)
        e = chat[:, None] * np.exp(-d / (2.0 * s2))
        P = pi[:, None] * e / ((pi[:, None] * e).sum(axis=0) + eta / (1 - eta) * np.sum(pi * chat))
        np.testing.assert_allclose(es.P, P, rtol=1e-11, atol=1e-300)


def test_depth_confidence_hand_values():
    P = np.zeros((5, 3))
    P[:, 2] = [0.5, 1.0, 2.0, 0.2, 3.0]
    coef = (1e-3, 0.0, 2e-3)        # e(0.5) = 1.5e-3, e(1) = 3e-3, e(2) = 9e-3
    phi = O.depth_confidence(P, coef, 1.5e-3)
    np.testing.assert_allclose(phi, [1.0, 0.5, 1.0 / 6.0, 1.0, 1.5e-3 / 19e-3], rtol=1e-15)
    # linear term
    phi = O.depth_confidence(P, (0.0, 1e-3, 0.0), 0.5e-3)
    np.testing.assert_allclose(phi, [1.0, 0.5, 0.25, 1.0, 1.0 / 6.0], rtol=1e-15)


def test_confidence_priors_properties():
    rng = np.random.default_rng(4)
    phy = rng.uniform(0.05, 1.0, size=40)
    phx = rng.uniform(0.05, 1.0, size=30)
    pi, w = O.confidence_priors(phy, phx, 0.1)
    assert pi.sum() == pytest.approx(1.0, rel=1e-15)
    np.testing.assert_allclose(pi / phy, pi[0] / phy[0], rtol=1e-14)   # pi proportional to phi
    assert np.all(w >= 0.1 - 1e-15) and np.all(w < 1.0)
    order = np.argsort(phx)
    assert np.all(np.diff(w[order]) <= 0)         # less confident => larger w_n
    pi1, w1 = O.confidence_priors(np.ones(40), np.ones(30), 0.1)
    np.testing.assert_allclose(pi1, 1.0 / 40, rtol=1e-15)
    np.testing.assert_allclose(w1, 0.1, rtol=1e-15)


def test_truncate_brute_force():
    rng = np.random.default_rng(5)
    P = rng.normal(size=(200, 3)).astype(np.float32)
    phi = rng.uniform(0, 1, size=200).astype(np.float32)
    thr = float(phi[7])                 # a tie: point 7 is kept
    Pk, fk = O.truncate(P, phi, thr)
    want = [i for i in range(200) if float(phi[i]) >= thr]
    assert 7 in want
    np.testing.assert_array_equal(Pk, P[want])
    np.testing.assert_array_equal(fk, phi[want])


def test_register_with_unit_confidences_is_plain_register():
    rng = datagen.rng_for(11, 0)
    p = datagen.scene_pair(rng, 300, 250, max_angle_deg=20.0)
    a = O.register(p.X, p.Y, k=10, max_iter=15)
    b = O.register(p.X, p.Y, k=10, max_iter=15, phi_x=np.ones(250), phi_y=np.ones(300),
                   cf_threshold=0.5)
    assert b.N == 250 and b.M == 300
    # w_n = 1 - (1 - w0) differs from w0 by an ulp; nothing else changes
    np.testing.assert_allclose(b.R, a.R, atol=1e-10)
    np.testing.assert_allclose(b.sigma2, a.sigma2, rtol=1e-9)
    np.testing.assert_allclose(b.nll, a.nll, rtol=1e-12)


def test_register_eta_and_confidence_filtering_recover_the_pose():
    p = datagen.depth_pair(trial=1, M=400, N=400)
    phx = O.depth_confidence(p.X, datagen.DEPTH_ERROR, datagen.DEPTH_ERROR_MIN)
    phy = O.depth_confidence(p.Y, datagen.DEPTH_ERROR, datagen.DEPTH_ERROR_MIN)
    r = O.register(p.X, p.Y, k=10, max_iter=40, eta=0.1, phi_x=phx, phi_y=phy,
                   cf_threshold=0.05)
    assert r.N == int(np.sum(phx >= 0.05)) and r.M == int(np.sum(phy >= 0.05))
    assert r.N < 400 and r.M < 400
    # 10 degrees apart at the start; a few hundred noisy points fix the pose
    # to a degree or two
    assert O.rotation_error_deg(r.R, p.R_gt) < 5.0
    # w0 = w_max at the initial sigma^2, from the kept points
    pi, _ = O.confidence_priors(phy[phy >= 0.05], None, 0.1)
    s2 = O.sigma2_init(p.X[phx >= 0.05], p.Y[phy >= 0.05], np.eye(3), np.zeros(3))
    assert r.w0 == O.outlier_weight_max(0.1, r.V, pi, r.alpha, s2)
    assert 0.0 < r.w0 < 0.5
