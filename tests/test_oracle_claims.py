"""The oracle against the paper's qualitative claims on synthetic data
(Sec. 4.1, registration on data with outliers and noise):

* the mean penalty alpha of the target falls as the points get noisier (the
  local surface looks less like a plane, Eq. 3), strictly, over noise levels
  from 0 to 3 % of the box diagonal;
* with as many Gaussian outliers as points in both clouds, LSG-CPD with w0
  from the outlier ratio (Sec. 3.2) still recovers the pose to under a degree,
  and more closely than the isotropic method (alpha_max = 0, i.e. rigid CPD)
  does on the same clouds;
* on a clean pair it stops on the same tolerance in fewer EM iterations than
  the isotropic method, at a smaller error.

These claims hold for the method, not for one implementation: a dropped plane
term, a wrong sign in it or an outlier weight that ignores eta breaks them."""
import numpy as np

import datagen
from oracle import lsgcpd_oracle as O


def test_mean_alpha_falls_with_noise():
    p = datagen.range_scanner_pair(trial=1, M=1500, N=1500, angle_deg=20.0)
    Y = p.Y.astype(np.float64)
    diag = O.bbox_diag(Y)
    rng = np.random.default_rng(3)
    means = []
    for s in (0.0, 0.005, 0.01, 0.02, 0.03):
        Yn = Y + rng.normal(scale=s * diag, size=Y.shape)
        _, _, alpha = O.normals(Yn, 20, 30.0, 0.2)
        means.append(float(np.mean(alpha)))
    assert all(a > b for a, b in zip(means, means[1:])), means
    assert means[0] > 25.0 and means[-1] < 0.5 * means[0], means


def test_outlier_ratio_one_recovers_and_beats_isotropic():
    q = datagen.range_scanner_pair(trial=2, M=400, N=400, angle_deg=20.0)
    X, Y = q.X.astype(np.float64), q.Y.astype(np.float64)
    rng = np.random.default_rng(3)
    lo, hi = Y.min(0), Y.max(0)
    c, spread = (lo + hi) / 2, (hi - lo) / 4
    Xo = np.vstack([X, rng.normal(c, spread, size=X.shape)]).astype(np.float32)
    Yo = np.vstack([Y, rng.normal(c, spread, size=Y.shape)]).astype(np.float32)
    lsg = O.register(Xo, Yo, k=10, max_iter=50, eta=0.5)
    iso = O.register(Xo, Yo, k=10, max_iter=50, eta=0.5, alpha_max=0.0)
    e_lsg = O.rotation_error_deg(lsg.R, q.R_gt)
    e_iso = O.rotation_error_deg(iso.R, q.R_gt)
    assert e_lsg < 1.0, e_lsg
    assert O.translation_error(lsg.t, q.t_gt) < 0.01 * O.bbox_diag(Y)
    assert e_lsg < e_iso, (e_lsg, e_iso)


def test_fewer_iterations_than_isotropic():
    q = datagen.range_scanner_pair(trial=2, M=400, N=400, angle_deg=20.0)
    lsg = O.register(q.X, q.Y, k=10, max_iter=300, tol=1e-6)
    iso = O.register(q.X, q.Y, k=10, max_iter=300, tol=1e-6, alpha_max=0.0)
    assert max(lsg.iters, iso.iters) < 300   # both stopped on the tolerance
    assert lsg.iters < iso.iters, (lsg.iters, iso.iters)
    assert O.rotation_error_deg(lsg.R, q.R_gt) < O.rotation_error_deg(iso.R, q.R_gt)
