"""The C form of the oracle's E step, kNN and initial variance (estep_ref.c)
against the NumPy oracle on small clouds (CPU)."""
import numpy as np
import pytest

import datagen
from oracle import c_oracle as CO
from oracle import lsgcpd_oracle as O


@pytest.fixture(scope="module", autouse=True)
def _built():
    CO.build()


@pytest.mark.parametrize("exact", [False, True])
def test_c_estep_columns_match_numpy(exact):
    p = datagen.range_scanner_pair(trial=7, M=350, N=280)
    n, _, a = O.normals(p.Y, 10, 30.0, 0.2)
    n32, a32 = n.astype(np.float32), a.astype(np.float32)
    rng = np.random.default_rng(0)
    w = rng.uniform(0.05, 0.5, size=280)
    pi = rng.uniform(0.5, 1.5, size=350)
    pi /= pi.sum()
    R, t = p.R_gt, p.t_gt + 0.01
    for s2 in (2e-4, 0.03):
        es = O.estep(p.X, p.Y, n32, a32, R, t, s2, V=2.5, pi=pi, w=w, exact_normalizer=exact)
        cols = O.columns(es.P, p.X, p.Y, n32, a32, R, t)
        cc, ks = CO.estep_columns(p.X, p.Y, n32, a32, R, t, s2, V=2.5, pi=pi, w=w,
                                  exact_normalizer=exact)
        np.testing.assert_allclose(ks, es.Ksum, rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(cc.p, cols.p, rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(cc.A, cols.A, rtol=1e-11, atol=1e-12 * np.abs(cols.A).max())
        np.testing.assert_allclose(cc.B, cols.B, rtol=1e-11, atol=1e-12 * np.abs(cols.B).max())
        np.testing.assert_allclose(cc.C, cols.C, rtol=1e-11, atol=1e-12 * np.abs(cols.C).max())
        np.testing.assert_allclose(cc.c, cols.c, rtol=1e-11, atol=1e-14)
    sub = np.array([5, 0, 279, 17])
    cs, ks2 = CO.estep_columns(p.X, p.Y, n32, a32, R, t, 0.03, V=2.5, pi=pi, w=w,
                               exact_normalizer=exact, sources=sub)
    np.testing.assert_allclose(ks2, ks[sub], rtol=1e-15)


def test_c_knn_and_sigma2_match_numpy():
    rng = np.random.default_rng(3)
    g = np.stack(np.meshgrid(np.arange(6), np.arange(5), np.arange(4), indexing="ij"), -1)
    Y = np.vstack([g.reshape(-1, 3) * 0.1, rng.normal(size=(150, 3))]).astype(np.float32)
    for k in (1, 7, 20):
        np.testing.assert_array_equal(CO.knn_indices(Y, k), O.knn_indices(Y, k))
    q = np.array([3, 100, 0])
    np.testing.assert_array_equal(CO.knn_indices(Y, 9, q), O.knn_indices(Y, 9, q))
    X = rng.normal(size=(90, 3)).astype(np.float32)
    R = datagen.random_rotation(rng, 0.4)
    assert CO.sigma2_init(X, Y, R, [0.1, 0, 0]) == pytest.approx(
        O.sigma2_init(X, Y, R, [0.1, 0, 0]), rel=1e-12)


def test_register_with_c_estep_equals_dense():
    p = datagen.range_scanner_pair(trial=8, M=260, N=240)
    n, _, a = O.normals(p.Y, 10, 30.0, 0.2)
    V = O.working_volume(p.Y)
    d = O.register(p.X, p.Y, max_iter=12, target_normals=n.astype(np.float32),
                   target_alpha=a.astype(np.float32))
    c = O.register(p.X, p.Y, max_iter=12, target_normals=n.astype(np.float32),
                   target_alpha=a.astype(np.float32),
                   estep_columns=CO.register_columns_fn(p.X, p.Y, n, a, 0.1, V))
    assert O.rotation_error_deg(c.R, d.R) < 1e-9
    np.testing.assert_allclose(c.nll, d.nll, rtol=1e-11)


def test_register_with_c_estep_and_confidences_equals_dense():
    # confidence filtering through the C E step (per-point priors and outlier
    # weights) against the NumPy oracle's own confidence filtering
    p = datagen.depth_pair(trial=5, M=260, N=240)
    phx = O.depth_confidence(p.X, datagen.DEPTH_ERROR, datagen.DEPTH_ERROR_MIN).astype(np.float32)
    phy = O.depth_confidence(p.Y, datagen.DEPTH_ERROR, datagen.DEPTH_ERROR_MIN).astype(np.float32)
    o = O.register(p.X, p.Y, k=10, max_iter=8, eta=0.1, phi_x=phx, phi_y=phy)
    pi, _ = O.confidence_priors(phy, None, 0.1)
    w0 = O.outlier_weight_max(0.1, o.V, pi, o.alpha, O.sigma2_init(p.X, p.Y, np.eye(3), np.zeros(3)))
    _, w = O.confidence_priors(None, phx, w0)
    n32, a32 = o.normals.astype(np.float32), o.alpha.astype(np.float32)
    fn = CO.register_columns_fn(p.X, p.Y, n32, a32, w0, o.V, pi=pi, w=w)
    c = O.register(p.X, p.Y, max_iter=8, target_normals=n32, target_alpha=a32, V=o.V,
                   estep_columns=fn)
    assert o.w0 == w0
    assert O.rotation_error_deg(c.R, o.R) < 1e-6
    np.testing.assert_allclose(c.nll, o.nll, rtol=1e-7)
