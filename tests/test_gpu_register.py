"""GPU parity of the target geometry (lsgcpd_normals) and of full
registrations (lsgcpd_register) against the FP64 oracle.

Bar: kappa and alpha within float32 output rounding, n n^T where the
eigengap is clear; registration: rotation <= 1e-3 deg, translation <=
1e-5 * box diagonal, the same number of EM iterations, NLL per iteration
within 1e-6 relative.
"""
import math

import numpy as np
import pytest

import datagen
from oracle import lsgcpd_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2103_15039_amd")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _check_normals(Y32, k, queries=None, amax=30.0, lam=0.2):
    n_g, k_g, a_g = L.normals(dev(Y32), k, amax, lam)
    n_g, k_g, a_g = (x.double().cpu().numpy() for x in (n_g, k_g, a_g))
    nbr = O.knn_indices(Y32, k, queries)
    n_o, k_o, lam_o, tr_o = O.local_geometry(Y32, nbr)
    a_o = O.penalty_alpha(k_o, amax, lam)
    q = np.arange(len(Y32)) if queries is None else np.asarray(queries)
    np.testing.assert_allclose(k_g[q], k_o, rtol=2e-6, atol=1e-9)
    np.testing.assert_allclose(a_g[q], a_o, rtol=2e-6, atol=1e-6 * amax)
    gap = (lam_o[:, 1] - lam_o[:, 0]) > 1e-3 * np.maximum(tr_o, 1e-300)
    dots = np.abs(np.sum(n_g[q] * n_o, axis=1))
    assert np.all(dots[gap] > 1 - 1e-6)
    return n_g, k_g, a_g


@pytest.mark.parametrize("M,k", [(1, 1), (7, 7), (300, 10), (2000, 10), (2000, 20), (5000, 32)])
def test_normals_parity(M, k):
    p = datagen.range_scanner_pair(trial=M, M=M, N=10)
    _check_normals(p.Y, k)


def test_normals_degenerate_inputs():
    rng = np.random.default_rng(3)
    Y = np.vstack([np.zeros((12, 3)), datagen.plane_patch(rng, 200, normal=(0, 1, 1)),
                   np.tile([[0.3, 0.2, 0.1]], (5, 1))]).astype(np.float32)
    n_g, k_g, a_g = _check_normals(Y, 10)
    assert np.allclose(k_g[:12], 1.0 / 3.0) and np.allclose(a_g[:12], 0.0)
    assert np.allclose(n_g[:12], [0, 0, 1])


def test_normals_rgbd_sampled():
    p = datagen.rgbd_pair()
    q = np.random.default_rng(0).choice(len(p.Y), size=300, replace=False)
    _check_normals(p.Y, 20, q)


@pytest.mark.parametrize("wl,k,nq", [("rgbd_20000x20000", 20, None), ("rgbd_20000x20000", 32, None),
                                     ("lidar_100000x50000", 20, 20000)])
def test_normals_full_size(wl, k, nq):
    """Every query (or 20,000 sampled ones) of the benchmark clouds: the tiled
    search with its target splits, hard queries (the RGB-D cloud has 5%
    outliers) and merge must give exactly the brute-force neighbour sets."""
    p = datagen.WORKLOADS[wl]()
    q = None if nq is None else np.random.default_rng(1).choice(len(p.Y), size=nq, replace=False)
    _check_normals(p.Y, k, q)


def _reg_pair(p, k, max_iter, tol=0.0, exact=False):
    g = L.register(dev(p.X), dev(p.Y), k=k, max_iter=max_iter, tol=tol, exact=exact)
    o = O.register(p.X, p.Y, k=k, max_iter=max_iter, tol=tol, exact_normalizer=exact)
    diag = O.bbox_diag(p.Y)
    assert g.iters == o.iters
    assert O.rotation_error_deg(g.R, o.R) <= 1e-3
    assert O.translation_error(g.t, o.t) <= 1e-5 * diag
    np.testing.assert_allclose(g.nll, o.nll, rtol=1e-6, atol=1e-6 * len(p.X))
    assert g.sigma2 == pytest.approx(o.sigma2, rel=1e-3)
    return g, o


def test_register_range_scanner_2000():
    p = datagen.range_scanner_pair(trial=0)
    g, o = _reg_pair(p, 10, 50)
    assert O.rotation_error_deg(g.R, p.R_gt) < 1.0


@pytest.mark.parametrize("trial", [1, 2])
def test_register_small_variants(trial):
    p = datagen.range_scanner_pair(trial=trial, M=600, N=450, angle_deg=20.0)
    _reg_pair(p, 10, 30, exact=(trial == 2))


def test_register_tol_stop_and_backends():
    p = datagen.range_scanner_pair(trial=3, M=500, N=500)
    g = L.register(dev(p.X), dev(p.Y), k=10, max_iter=60, tol=1e-7)
    o = O.register(p.X, p.Y, k=10, max_iter=60, tol=1e-7)
    assert g.converged and g.iters == o.iters < 60
    # dense keeps the caller's source order; the default sorts sources
    # spatially, which changes only the rounding of the sums
    d = L.register(dev(p.X), dev(p.Y), k=10, max_iter=60, tol=1e-7, backend="dense")
    assert d.iters == g.iters and O.rotation_error_deg(d.R, g.R) < 1e-7
    # the two sum the same terms in different groupings; over ~40 EM
    # iterations that leaves the NLL traces ~1e-12 apart
    np.testing.assert_allclose(d.nll, g.nll, rtol=1e-11)
    for backend in ("lds", "mfma"):
        v = L.register(dev(p.X), dev(p.Y), k=10, max_iter=60, tol=1e-7, backend=backend)
        assert v.iters == g.iters
        assert O.rotation_error_deg(v.R, g.R) < 1e-5


def test_register_nll_monotone_and_recovery():
    rng = np.random.default_rng(21)
    Y = datagen._sample_box_sphere(rng, 1500)
    Rg = datagen.random_rotation(rng, math.radians(25.0))
    tg = rng.uniform(-0.1, 0.1, size=3)
    X = ((Y - tg) @ Rg).astype(np.float32)
    g = L.register(dev(X), dev(Y.astype(np.float32)), k=10, max_iter=100)
    assert np.all(np.diff(g.nll) <= 1e-7 * np.abs(g.nll[1:]))
    assert O.rotation_error_deg(g.R, Rg) < 1e-3
    assert O.translation_error(g.t, tg) < 1e-5 * O.bbox_diag(Y)


def test_autotune_picks_a_candidate_and_keeps_parity():
    p = datagen.range_scanner_pair(trial=6, M=2000, N=1800, angle_deg=20.0)
    best = L.autotune(dev(p.X), dev(p.Y), k=10, max_iter=20)
    assert best in (1024, 2048, 4096, 8192, 16384, 32768)
    g, _ = _reg_pair(p, 10, 20)
    again = L.register(dev(p.X), dev(p.Y), k=10, max_iter=20)
    assert np.array_equal(again.R, g.R) and np.array_equal(again.nll, g.nll)
