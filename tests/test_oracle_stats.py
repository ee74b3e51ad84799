"""Pins for the oracle's 86 lifted statistics (the reference for every GPU
statistic) and for the registration error of Eq. (14).

The statistics are pinned by what they are for: Q of Eq. (6) at any pose is a
fixed quadratic in the 12 entries of G = [R | t], and the statistics are its
coefficients.  So D(G) assembled from them must equal the dense double sum
sum_mn P_mn d_mn(G) over the posterior at an arbitrary 3 x 4 matrix G (not
only at rotations), with d_mn the Mahalanobis form of Eq. (2), written out here
as a loop over pairs.  Its derivatives along SE(3) must equal Eq. (11)-(12) as
printed.  A transposed block, a wrong triangle order or a dropped term changes
D at a random G, so each of those mistakes fails here.
"""
import math

import numpy as np
import pytest

import datagen
from oracle import lsgcpd_oracle as O

IU4 = [(i, j) for i in range(4) for j in range(i, 4)]      # 00 01 02 03 11 12 13 22 23 33
IU3 = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def _sym4(v):
    S = np.zeros((4, 4))
    for k, (i, j) in enumerate(IU4):
        S[i, j] = S[j, i] = v[k]
    return S


def _D_from_stats(s, G):
    """D(G) = sum_a G_a^T S0 G_a + sum_ab G_a^T S1[a,b] G_b - 2 sum_a S2[a].G_a + S3
    with G_a the a-th row of G (4 entries) and S1[b,a] = S1[a,b]."""
    S0 = _sym4(s[0:10])
    S1 = {}
    for k, (a, b) in enumerate(IU3):
        S1[(a, b)] = S1[(b, a)] = _sym4(s[10 + 10 * k:20 + 10 * k])
    S2 = s[70:82].reshape(3, 4)
    D = s[82]
    for a in range(3):
        D += G[a] @ S0 @ G[a] - 2.0 * S2[a] @ G[a]
        for b in range(3):
            D += G[a] @ S1[(a, b)] @ G[b]
    return float(D)


def _D_dense(P, X, Y, nrm, alpha, G):
    """sum_mn P_mn (G x~_n - y_m)^T (I + alpha_m n_m n_m^T) (G x~_n - y_m), pair by pair."""
    tot = 0.0
    for m in range(Y.shape[0]):
        Mm = np.eye(3) + alpha[m] * np.outer(nrm[m], nrm[m])
        for n in range(X.shape[0]):
            r = G[:, :3] @ X[n] + G[:, 3] - Y[m]
            tot += P[m, n] * float(r @ Mm @ r)
    return tot


def _problem(seed, M, N, per_point=False):
    rng = np.random.default_rng(seed)
    Y = rng.normal(size=(M, 3)) * 0.6 + rng.normal(size=3)
    X = Y[rng.integers(0, M, size=N)] + rng.normal(size=(N, 3)) * 0.2
    nrm = rng.normal(size=(M, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    alpha = rng.uniform(0.5, 25.0, size=M)
    R = datagen.random_rotation(rng, 0.3)
    t = rng.normal(size=3) * 0.1
    pi = w = None
    if per_point:
        pi = rng.uniform(0.2, 1.0, size=M)
        pi /= pi.sum()
        w = rng.uniform(0.05, 0.8, size=N)
    return rng, X, Y, nrm, alpha, R, t, pi, w


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("per_point", [False, True])
@pytest.mark.parametrize("seed,M,N", [(0, 15, 12), (1, 9, 20)])
def test_stats_reproduce_dense_quadratic(seed, M, N, per_point, exact):
    rng, X, Y, nrm, alpha, R, t, pi, w = _problem(seed, M, N, per_point)
    s2 = 0.3
    es = O.estep(X, Y, nrm, alpha, R, t, s2, w0=0.1, V=4.0, pi=pi, w=w,
                 exact_normalizer=exact)
    cols = O.columns(es.P, X, Y, nrm, alpha, R, t)
    s = O.lifted_stats(cols, X, O.nll_terms(es, w, 0.1))
    for trial in range(6):
        G = rng.normal(size=(3, 4)) * (0.3 if trial else 0.0)   # trial 0: G = 0 gives S3
        if trial == 1:
            G = np.hstack([R, t[:, None]])
        ref = _D_dense(es.P, X, Y, nrm, alpha, G)
        got = _D_from_stats(s, G)
        assert got == pytest.approx(ref, rel=1e-12, abs=1e-13)


def test_stats_each_block_matters():
    """A plausible packing mistake moves D at a random G (the identity above is
    not blind to it)."""
    rng, X, Y, nrm, alpha, R, t, _, _ = _problem(3, 10, 11)
    es = O.estep(X, Y, nrm, alpha, R, t, 0.3, w0=0.1, V=4.0)
    cols = O.columns(es.P, X, Y, nrm, alpha, R, t)
    s = O.lifted_stats(cols, X)
    G = rng.normal(size=(3, 4))
    ref = _D_dense(es.P, X, Y, nrm, alpha, G)
    bad = []
    s2t = s.copy()
    s2t[70:82] = s[70:82].reshape(4, 3).T.reshape(12)              # S2 read as 4 x 3
    bad.append(s2t)
    swap = s.copy()
    swap[10:20], swap[20:30] = s[20:30], s[10:20]                  # S1[00] <-> S1[01]
    bad.append(swap)
    tri = s.copy()
    tri[1], tri[4] = s[4], s[1]                                    # S0: 01 <-> 11
    bad.append(tri)
    drop = s.copy()
    drop[82] = 0.0
    bad.append(drop)
    for b in bad:
        assert abs(_D_from_stats(b, G) - ref) > 1e-6 * abs(ref)


@pytest.mark.parametrize("seed", [0, 4])
def test_stats_derivatives_are_eq11_12(seed):
    """D(G0 exp(xi^)) / sigma^2 from the statistics has the gradient and the
    symmetrised Hessian of Eq. (11)-(12) as printed (double sums over pairs)."""
    rng, X, Y, nrm, alpha, R, t, pi, w = _problem(seed, 12, 10, per_point=True)
    s2 = 0.05
    es = O.estep(X, Y, nrm, alpha, R, t, s2, w0=0.1, V=3.0, pi=pi, w=w)
    cols = O.columns(es.P, X, Y, nrm, alpha, R, t)
    s = O.lifted_stats(cols, X)
    g0 = O.homog(R, t)
    f = lambda xi: _D_from_stats(s, (g0 @ O.se3_exp(xi))[:3]) / s2
    grad, H = O.grad_hess_literal(es.P, X, Y, nrm, alpha, R, t, s2)
    h = 1e-5
    E6 = np.eye(6)
    fd = np.array([(f(h * E6[i]) - f(-h * E6[i])) / (2 * h) for i in range(6)])
    np.testing.assert_allclose(fd, grad, rtol=1e-7, atol=1e-7 * np.abs(grad).max())
    Hfd = np.empty((6, 6))
    for i in range(6):
        for j in range(6):
            Hfd[i, j] = (f(h * (E6[i] + E6[j])) - f(h * (E6[i] - E6[j]))
                         - f(h * (E6[j] - E6[i])) + f(-h * (E6[i] + E6[j]))) / (4 * h * h)
    Hs = 0.5 * (H + H.T)
    np.testing.assert_allclose(Hfd, Hs, rtol=1e-4, atol=1e-4 * np.abs(Hs).max())


@pytest.mark.parametrize("per_point", [False, True])
def test_stats_nll_terms(per_point):
    """Entries 83-85 give Eq. (4)'s negative log-likelihood (which is pinned to
    scipy's Gaussian densities elsewhere) and the outlier mass N - sum_mn P_mn."""
    rng, X, Y, nrm, alpha, R, t, pi, w = _problem(7, 13, 17, per_point)
    s2 = 0.08
    es = O.estep(X, Y, nrm, alpha, R, t, s2, w0=0.2, V=5.0, pi=pi, w=w)
    cols = O.columns(es.P, X, Y, nrm, alpha, R, t)
    s = O.lifted_stats(cols, X, O.nll_terms(es, w, 0.2))
    N = X.shape[0]
    nll = -(s[85] + s[83] - 1.5 * N * math.log(2 * math.pi * s2))
    assert nll == pytest.approx(es.nll, rel=1e-13)
    assert s[84] == pytest.approx(N - float(np.sum(es.P)), rel=1e-12)
    # S0[3,3] (entry 9) is N_P = sum_mn P_mn
    assert s[9] == pytest.approx(float(np.sum(es.P)), rel=1e-13)


def test_registration_error_eq14_hand_values():
    """Eq. (14): mean over source points of |g(x_i) - g_gt(x_i)|."""
    X = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 2.0, 0.0]])
    Rz90 = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    # g rotates by 90 deg about z, g_gt is the identity:
    # (1,0,0) -> (0,1,0): sqrt(2);  (0,0,1) fixed: 0;  (0,2,0) -> (-2,0,0): 2 sqrt(2)
    e = O.registration_error(X, Rz90, np.zeros(3), np.eye(3), np.zeros(3))
    assert e == pytest.approx((math.sqrt(2) + 0.0 + 2 * math.sqrt(2)) / 3, rel=1e-15)
    # equal rotations, translations 3 apart: every point is 3 off
    e = O.registration_error(X, Rz90, np.array([1.0, 2.0, 2.0]), Rz90, np.zeros(3))
    assert e == pytest.approx(3.0, rel=1e-15)
    # identical transforms: 0
    assert O.registration_error(X, Rz90, np.ones(3), Rz90, np.ones(3)) == 0.0
