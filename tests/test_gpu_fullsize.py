"""GPU parity at the workloads' full sizes (20,000 x 20,000 RGBD-like and
100,000 x 50,000 LiDAR-like), in the launch configuration the benchmark uses.

* one E step: every statistic against the C form of the oracle over all
  M x N pairs; per-source sums of a random sample of sources against the
  dense NumPy oracle; the column identity for every source;
* registration: the 20k pair for its whole 50 EM iterations, and the
  100k x 50k pair for 3 iterations from the identity and 5 from its ground
  truth at a small sigma^2, against the oracle driven by the C E step
  (rotation <= 1e-3 deg, translation <= 1e-5 * box diagonal, NLL per
  iteration 1e-6); after the runs that end in the converged regime, one E
  step at the oracle's final pose and sigma^2 with all 86 statistics against
  the C oracle.
Normals for the E-step checks are seeded random unit vectors and penalties
(an E step does not care where they come from); registrations compute their
own normals on each side.
"""
import numpy as np
import pytest

import datagen
from oracle import c_oracle as CO
from oracle import lsgcpd_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2103_15039_amd")

_PAIRS = {}


def pair(name):
    if name not in _PAIRS:
        _PAIRS[name] = {"rgbd": datagen.rgbd_pair, "lidar": datagen.lidar_pair}[name]()
    return _PAIRS[name]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.fixture(scope="module", autouse=True)
def _c_oracle():
    CO.build()


def _geometry(M, seed):
    rng = np.random.default_rng(seed)
    n = rng.normal(size=(M, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return n.astype(np.float32), rng.uniform(0.0, 30.0, size=M).astype(np.float32)


def _abs_scale(cols, X):
    W = cols.A - cols.p[:, None, None] * np.eye(3)[None]
    ab = O.Columns(p=np.abs(cols.p), A=np.abs(W) + np.abs(cols.p)[:, None, None] * np.eye(3)[None],
                   B=np.abs(cols.B), C=np.abs(cols.C), b=None, c=None)
    return O.lifted_stats(ab, np.abs(X))


@pytest.mark.parametrize("name,s2", [("rgbd", 2e-3), ("rgbd", 0.05), ("lidar", 5e-3),
                                     ("lidar", 0.2)])
def test_estep_full_size(name, s2):
    p = pair(name)
    M, N = len(p.Y), len(p.X)
    n32, a32 = _geometry(M, 1)
    rng = np.random.default_rng(2)
    R = datagen.random_rotation(rng, 0.01) @ p.R_gt
    t = p.t_gt + rng.uniform(-0.02, 0.02, size=3)
    V = O.working_volume(p.Y)
    g = L.estep(dev(p.X), dev(p.Y), dev(n32), dev(a32), R, t, s2, w0=0.1, colstats=True)
    assert g.V == pytest.approx(V, rel=1e-14)
    cs = g.colstats.cpu().numpy()
    # every column: components + outlier = 1
    np.testing.assert_allclose(cs[:, 2] + cs[:, 14], 1.0, rtol=0, atol=1e-12)
    assert g.sumP + g.outlier_mass == pytest.approx(N, rel=1e-12)
    # sampled columns against the dense oracle
    smp = np.sort(rng.choice(N, size=48, replace=False))
    es = O.estep(p.X[smp], p.Y, n32, a32, R, t, s2, w0=0.1, V=V)
    cols = O.columns(es.P, p.X[smp], p.Y, n32, a32, R, t)
    assert np.all(np.abs(cs[smp, 1] - es.Ksum) <= 1e-5 * (es.Ksum + es.gamma))
    np.testing.assert_allclose(cs[smp, 2], cols.p, rtol=1e-5, atol=1e-12)
    W = cols.A - cols.p[:, None, None] * np.eye(3)[None]
    iu = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    Wref = np.stack([W[:, a, b] for a, b in iu], axis=1)
    np.testing.assert_allclose(cs[smp, 3:9], Wref, rtol=1e-5,
                               atol=1e-5 * np.abs(Wref).max() + 1e-12)
    np.testing.assert_allclose(cs[smp, 9:12], cols.B, rtol=1e-5,
                               atol=1e-5 * np.abs(cols.B).max() + 1e-12)
    np.testing.assert_allclose(cs[smp, 12], cols.C, rtol=1e-5, atol=1e-12)
    # every statistic against the C oracle over all pairs
    cc, ks = CO.estep_columns(p.X, p.Y, n32, a32, R, t, s2, w0=0.1, V=V)
    gamma = (2 * np.pi * s2) ** 1.5 / V
    ref = O.lifted_stats(cc, p.X, [np.sum(np.log(ks + gamma)), np.sum(gamma / (ks + gamma)),
                                   N * np.log(0.1)])
    scale = _abs_scale(cc, p.X.astype(np.float64))
    scale[83:] = np.abs(ref[83:]) + N
    d = np.abs(g.stats - ref)
    bad = np.nonzero(d > 2e-6 * scale + 1e-300)[0]
    assert bad.size == 0, f"stats {bad[:8]}: gpu {g.stats[bad[:4]]} ref {ref[bad[:4]]}"


def _oracle_normals(Y, k):
    nbr = CO.knn_indices(Y, k)
    n, kappa, _, _ = O.local_geometry(Y, nbr)
    return n, O.penalty_alpha(kappa, 30.0, 0.2)


def _spatial_order(X, bits=10):
    """A permutation that lists the points cell by cell along a Z-order curve
    of a 2^bits grid over their box (numpy only): lsgcpd_estep takes the
    sources in the caller's order, and spatially coherent groups of sources
    let its exact culling work as it does inside a registration.  The
    statistics are sums over all sources, so any order gives them."""
    lo, hi = X.min(axis=0), X.max(axis=0)
    q = ((X - lo) / np.maximum(hi - lo, 1e-30) * ((1 << bits) - 1)).astype(np.uint64)
    key = np.zeros(len(X), np.uint64)
    for b in range(bits):
        for a in range(3):
            key |= ((q[:, a] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + a)
    return np.argsort(key, kind="stable")


def _stats_vs_c_oracle(p, n, a, R, t, s2, w0=0.1):
    """One GPU E step against the C oracle over all M x N pairs: every one of
    the 86 statistics within 2e-6 of the sum of the magnitudes of its terms
    (the float32 exponential's relative error, argument rounding included, is
    below 2e-6 wherever a term is not negligible), the NLL within 1e-6.
    Returns the fraction of pairs the GPU evaluated."""
    N, M = len(p.X), len(p.Y)
    V = O.working_volume(p.Y)
    p = datagen.Pair(X=np.ascontiguousarray(p.X[_spatial_order(p.X)]), Y=p.Y, R_gt=p.R_gt,
                     t_gt=p.t_gt)
    L.profile_enable(True)
    L.profile_read(reset=True)
    g = L.estep(dev(p.X), dev(p.Y), dev(n), dev(a), R, t, s2, w0=w0)
    prof = L.profile_read(reset=True)
    L.profile_enable(False)
    cc, ks = CO.estep_columns(p.X, p.Y, n, a, R, t, s2, w0=w0, V=V)
    gamma = (2 * np.pi * s2) ** 1.5 / V
    ref = O.lifted_stats(cc, p.X, [np.sum(np.log(ks + gamma)), np.sum(gamma / (ks + gamma)),
                                   N * np.log(w0)])
    scale = _abs_scale(cc, p.X.astype(np.float64))
    scale[83:] = np.abs(ref[83:]) + N
    d = np.abs(g.stats - ref)
    bad = np.nonzero(d > 2e-6 * scale + 1e-300)[0]
    assert bad.size == 0, f"stats {bad[:8]}: gpu {g.stats[bad[:4]]} ref {ref[bad[:4]]}"
    nll = -(ref[85] + ref[83] - 1.5 * N * np.log(2 * np.pi * s2))
    assert g.nll == pytest.approx(nll, rel=1e-6)
    return prof["evaluated_pairs"] / (M * N)


def _c_register(p, n, a, iters, R0=None, t0=None, s20=None):
    V = O.working_volume(p.Y)
    if s20 is None:
        s20 = CO.sigma2_init(p.X, p.Y, np.eye(3) if R0 is None else R0,
                             np.zeros(3) if t0 is None else t0)
    return O.register(p.X, p.Y, max_iter=iters, target_normals=n, target_alpha=a, V=V,
                      R0=R0, t0=t0, sigma2_0=s20,
                      estep_columns=CO.register_columns_fn(p.X, p.Y, n, a, 0.1, V))


def _check_registration(g, o, p, iters):
    diag = O.bbox_diag(p.Y)
    assert g.iters == o.iters == iters
    assert O.rotation_error_deg(g.R, o.R) <= 1e-3
    assert O.translation_error(g.t, o.t) <= 1e-5 * diag
    np.testing.assert_allclose(g.nll, o.nll, rtol=1e-6)
    assert g.sigma2 == pytest.approx(o.sigma2, rel=1e-4)


def test_register_rgbd_full_run_and_final_estep():
    """The RGB-D pair's whole 50-iteration registration against the oracle
    driven by the C E step; then one E step at the pose and sigma^2 the
    oracle's registration ends on (the late regime, where the exact culling
    drops most pairs), all 86 statistics against the C oracle."""
    p = pair("rgbd")
    k, iters = 20, 50
    g = L.register(dev(p.X), dev(p.Y), k=k, max_iter=iters)
    n, a = _oracle_normals(p.Y, k)
    o = _c_register(p, n, a, iters)
    _check_registration(g, o, p, iters)
    frac = _stats_vs_c_oracle(p, n.astype(np.float32), a.astype(np.float32), o.R, o.t, o.sigma2)
    assert frac < 0.5   # the check covered the culled regime


def test_register_lidar_from_truth_and_final_estep():
    """The LiDAR pair started at its ground-truth pose with sigma^2_0 = 0.05:
    5 EM iterations against the oracle driven by the C E step reach the
    converged regime; then one E step at the oracle's final pose and sigma^2,
    all 86 statistics against the C oracle."""
    p = pair("lidar")
    k, iters = 20, 5
    g = L.register(dev(p.X), dev(p.Y), k=k, max_iter=iters, R0=p.R_gt, t0=p.t_gt,
                   sigma2_init=0.05)
    n, a = _oracle_normals(p.Y, k)
    o = _c_register(p, n, a, iters, R0=p.R_gt, t0=p.t_gt, s20=0.05)
    _check_registration(g, o, p, iters)
    frac = _stats_vs_c_oracle(p, n.astype(np.float32), a.astype(np.float32), o.R, o.t, o.sigma2)
    assert frac < 0.5


def test_register_lidar_first_iterations():
    """The LiDAR pair from the identity, 3 EM iterations (the dense regime)."""
    p = pair("lidar")
    k, iters = 20, 3
    g = L.register(dev(p.X), dev(p.Y), k=k, max_iter=iters)
    n, a = _oracle_normals(p.Y, k)
    _check_registration(g, _c_register(p, n, a, iters), p, iters)


def test_register_cf_full_size():
    """Confidence filtering with truncation and w0 from the outlier ratio on
    a full-size depth-camera pair (20,000 x 20,000 before truncation): the
    kept points, w0 and 10 EM iterations against the oracle driven by the C E
    step with the same priors and outlier weights."""
    p = datagen.depth_pair(trial=0)
    conf = lambda P: O.depth_confidence(P, datagen.DEPTH_ERROR,
                                        datagen.DEPTH_ERROR_MIN).astype(np.float32)
    phx, phy = conf(p.X), conf(p.Y)
    thr, eta, iters, k = 0.05, 0.1, 10, 20
    g = L.register_cf(dev(p.X), dev(p.Y), dev(phx), dev(phy), threshold=thr, k=k,
                      max_iter=iters, eta=eta)
    Xk, fx = O.truncate(p.X, phx, thr)
    Yk, fy = O.truncate(p.Y, phy, thr)
    assert (g.n_used, g.m_used) == (len(Xk), len(Yk))
    n, a = _oracle_normals(Yk, k)
    V = O.working_volume(Yk)
    s20 = CO.sigma2_init(Xk, Yk, np.eye(3), np.zeros(3))
    pi, _ = O.confidence_priors(fy, None, 0.1)
    w0 = O.outlier_weight_max(eta, V, pi, a, s20)
    _, w = O.confidence_priors(None, fx, w0)
    o = O.register(Xk, Yk, max_iter=iters, target_normals=n, target_alpha=a, V=V,
                   sigma2_0=s20,
                   estep_columns=CO.register_columns_fn(Xk, Yk, n, a, w0, V, pi=pi, w=w))
    diag = O.bbox_diag(Yk)
    assert g.w0 == pytest.approx(w0, rel=1e-9)
    assert g.iters == o.iters == iters
    assert O.rotation_error_deg(g.R, o.R) <= 1e-3
    assert O.translation_error(g.t, o.t) <= 1e-5 * diag
    np.testing.assert_allclose(g.nll, o.nll, rtol=1e-6)
    assert g.sigma2 == pytest.approx(o.sigma2, rel=1e-4)


def test_estep_million_points():
    """Ten times the benchmark's size in each cloud (10^12 pairs per E step):
    the column identity for every source, and 64 sampled sources against the C
    oracle's columns over all 10^6 targets."""
    p = datagen.scene_pair(datagen.rng_for(14, 0), 1_000_000, 1_000_000, max_angle_deg=10.0)
    M, N = len(p.Y), len(p.X)
    n32, a32 = _geometry(M, 3)
    s2 = 1e-4
    V = O.working_volume(p.Y)
    g = L.estep(dev(p.X), dev(p.Y), dev(n32), dev(a32), p.R_gt, p.t_gt, s2, w0=0.1,
                colstats=True)
    cs = g.colstats.cpu().numpy()
    np.testing.assert_allclose(cs[:, 2] + cs[:, 14], 1.0, rtol=0, atol=1e-12)
    assert g.sumP + g.outlier_mass == pytest.approx(N, rel=1e-12)
    smp = np.sort(np.random.default_rng(4).choice(N, size=64, replace=False))
    cc, ks = CO.estep_columns(p.X, p.Y, n32, a32, p.R_gt, p.t_gt, s2, w0=0.1, V=V, sources=smp)
    gamma = (2 * np.pi * s2) ** 1.5 / V
    assert np.all(np.abs(cs[smp, 1] - ks) <= 1e-5 * (ks + gamma))
    np.testing.assert_allclose(cs[smp, 2], cc.p, rtol=1e-5, atol=1e-12)
    np.testing.assert_allclose(cs[smp, 9:12], cc.B, rtol=1e-5,
                               atol=1e-5 * np.abs(cc.B).max() + 1e-12)
    np.testing.assert_allclose(cs[smp, 12], cc.C, rtol=1e-5, atol=1e-12)
