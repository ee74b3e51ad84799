"""Pins for the oracle's target geometry: kNN, normals, surface variation,
penalty alpha (Sec. 3.1, Eq. 3)."""
import math

import numpy as np
import pytest

import datagen
from oracle import lsgcpd_oracle as O


def _knn_bruteforce(Y, k):
    """Independent brute force: Python loops and sorted() on (distance, index),
    distances rounded to float32 after every operation."""
    Y = np.asarray(Y, dtype=np.float32)
    out = []
    for q in range(Y.shape[0]):
        cand = []
        for j in range(Y.shape[0]):
            s = np.float32(0.0)
            acc = []
            for c in range(3):
                d = np.float32(Y[q, c] - Y[j, c])
                acc.append(np.float32(d * d))
            s = np.float32(np.float32(acc[0] + acc[1]) + acc[2])
            cand.append((float(s), j))
        cand.sort()
        out.append([j for _, j in cand[:k]])
    return np.array(out)


def test_knn_matches_bruteforce_with_ties():
    rng = np.random.default_rng(1)
    # a lattice has many exactly equal distances: exercises the tie rule
    g = np.stack(np.meshgrid(np.arange(4), np.arange(3), np.arange(2), indexing="ij"), -1)
    Y = np.vstack([g.reshape(-1, 3) * 0.25, rng.normal(size=(16, 3))]).astype(np.float32)
    for k in (1, 5, 10):
        np.testing.assert_array_equal(O.knn_indices(Y, k), _knn_bruteforce(Y, k))


def test_knn_includes_self_and_duplicates_by_index():
    Y = np.array([[0, 0, 0], [0, 0, 0], [1, 0, 0], [0, 0, 0]], np.float32)
    nb = O.knn_indices(Y, 3)
    # the three coincident points are each other's nearest, lowest index first
    np.testing.assert_array_equal(nb[3], [0, 1, 3])
    np.testing.assert_array_equal(nb[2], [2, 0, 1])


def test_normals_on_exact_plane():
    rng = np.random.default_rng(2)
    nrm = np.array([1.0, 2.0, -2.0]) / 3.0
    Y = datagen.plane_patch(rng, 200, normal=nrm, offset=0.3)
    n, kappa, alpha = O.normals(Y, 10, 30.0, 0.2)
    assert np.all(kappa < 1e-12)
    assert np.allclose(np.abs(n @ nrm), 1.0, atol=1e-9)
    assert np.allclose(alpha, 30.0, atol=1e-9)


def test_axis_neighbourhood_closed_form():
    # neighbourhood {0, +-a e1, +-b e2, +-c e3}: covariance diag(2a^2, 2b^2, 2c^2)/7
    for (a, b, c) in ((1.0, 1.0, 1.0), (1.0, 0.5, 0.25), (0.3, 2.0, 0.7)):
        Y = np.array([[0, 0, 0], [a, 0, 0], [-a, 0, 0], [0, b, 0], [0, -b, 0],
                      [0, 0, c], [0, 0, -c]], dtype=np.float64)
        nbr = np.tile(np.arange(7), (7, 1))
        n, kappa, lam, tr = O.local_geometry(Y, nbr)
        ev = np.array([2 * a * a, 2 * b * b, 2 * c * c]) / 7.0
        assert abs(kappa[0] - ev.min() / ev.sum()) < 1e-14
        assert abs(abs(n[0][np.argmin(ev)]) - 1.0) < 1e-12
        if a == b == c:
            assert abs(kappa[0] - 1.0 / 3.0) < 1e-14
            assert O.penalty_alpha(kappa[:1], 30.0, 0.2)[0] < 1e-12


def test_normals_rigid_motion_equivariant():
    rng = np.random.default_rng(3)
    p = datagen.range_scanner_pair(trial=3, M=300, N=10)
    Y = p.Y.astype(np.float64)
    Rr = datagen.random_rotation(rng, 0.7)
    nbr = O.knn_indices(Y, 10)
    n0, k0, _, _ = O.local_geometry(Y, nbr)
    n1, k1, _, _ = O.local_geometry(Y @ Rr.T + np.array([0.3, -2.0, 1.0]), nbr)
    assert np.allclose(k0, k1, atol=1e-12)
    gap_ok = np.ones(len(Y), bool)
    _, _, lam, tr = O.local_geometry(Y, nbr)
    gap_ok = (lam[:, 1] - lam[:, 0]) > 1e-6 * tr
    assert np.allclose(np.abs(np.sum((n0 @ Rr.T) * n1, axis=1))[gap_ok], 1.0, atol=1e-8)


def test_kappa_range_and_eigen_property():
    rng = np.random.default_rng(4)
    Y = rng.normal(size=(150, 3))
    nbr = O.knn_indices(Y, 12)
    n, kappa, lam, tr = O.local_geometry(Y, nbr)
    assert np.all(kappa >= 0) and np.all(kappa <= 1 / 3 + 1e-15)
    # n is the minimiser of the Rayleigh quotient: compare with random directions
    P = Y[nbr]
    D = P - P.mean(axis=1, keepdims=True)
    C = np.einsum("mki,mkj->mij", D, D) / 12
    rq_n = np.einsum("mi,mij,mj->m", n, C, n)
    for _ in range(20):
        v = rng.normal(size=(len(Y), 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        assert np.all(rq_n <= np.einsum("mi,mij,mj->m", v, C, v) + 1e-14)
    assert np.allclose(rq_n / np.trace(C, axis1=1, axis2=2), kappa, atol=1e-14)


def test_alpha_tanh_identity_and_limits():
    kappa = np.concatenate([[0.0, 1e-300, 1e-6], np.linspace(0.001, 1 / 3, 200)])
    for amax, lam in ((30.0, 0.2), (1.0, 1.0), (100.0, 0.05)):
        a = O.penalty_alpha(kappa, amax, lam)
        with np.errstate(divide="ignore"):
            ref = amax * np.tanh(lam * (1.0 / kappa - 3.0) / 2.0)
        assert np.allclose(a, np.maximum(ref, 0), rtol=1e-13, atol=1e-13)
        assert a[0] == amax
        assert abs(a[-1]) < 1e-12 * amax            # kappa = 1/3 -> 0
        assert np.all(np.diff(a[3:]) <= 1e-12)      # decreasing in kappa


def test_alpha_table_at_default_parameters():
    # alpha / alpha_max at lambda = 0.2 for kappa = 0.01, 0.05, 0.1, 0.2, 0.3
    a = O.penalty_alpha(np.array([0.01, 0.05, 0.1, 0.2, 0.3]), 1.0, 0.2)
    expect = [math.tanh(0.1 * (1 / k - 3)) for k in (0.01, 0.05, 0.1, 0.2, 0.3)]
    assert np.allclose(a, expect, rtol=1e-14)
    assert np.allclose(a, [1.0, 0.94, 0.60, 0.20, 0.03], atol=0.01)


def test_working_volume_and_sigma2_init():
    Y = np.array([[0, 0, 0], [2, 1, 0.5], [1, 0.5, 0.25]], float)
    assert O.working_volume(Y) == pytest.approx(1.0)
    Yf = np.array([[0, 0, 0], [1, 1, 0]], float)          # flat: z edge floored
    assert O.working_volume(Yf) == pytest.approx(1e-3 * math.sqrt(2))
    rng = np.random.default_rng(5)
    X, Y = rng.normal(size=(7, 3)), rng.normal(size=(5, 3))
    s = sum(np.sum((x - y) ** 2) for x in X for y in Y) / (3 * 35)
    assert O.sigma2_init(X, Y, np.eye(3), np.zeros(3)) == pytest.approx(s, rel=1e-14)
