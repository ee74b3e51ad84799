"""Pins of the proposal oracle (oracle/proposal_ref.py) against what the
mathematics fixes, on the CPU:
  * Gram-Schmidt: orthonormal with determinant +1, the identity from
    (e_x, e_y), equivariance R(Q a1, Q a2) = Q R(a1, a2), invariance to a
    positive scale of a1 and to adding a multiple of a1 to a2;
  * the forward pass against an independent float64 implementation written
    with torch's own layers (nn.functional.linear, relu, amax);
  * every gradient of the batch loss against central finite differences,
    and the loss as least squares on the 6-D outputs (a half-turn label
    still pulls);
  * Adam: the first update is -lr * g / (|g| + eps) in closed form, and a
    second one against the published recurrences evaluated by hand;
  * normalisation and the pose mapping: a round trip through normalised
    units returns the pose, the sampled indices are evenly spaced, and the
    principal-axis frames are the eigenvectors of the covariance in the
    stated order and signs, rotating with the points.
A plausible mistake anywhere (a transposed weight, the source and target
features swapped, a missing ReLU mask, a target column taken as a row, an
unbiased Adam) fails one of these.
"""
import numpy as np
import pytest

import datagen
from oracle import proposal_ref as PR

torch = pytest.importorskip("torch")


def test_parameter_count():
    assert PR.NPARAM == 64 * 3 + 64 + 128 * 64 + 128 + 256 * 128 + 256 + 128 * 512 + 128 + 9 * 128 + 9
    assert PR.NPARAM == 108425


def test_gram_schmidt_properties():
    rng = np.random.default_rng(0)
    assert np.allclose(PR.gram_schmidt(np.array([1.0, 0, 0]), np.array([0, 1.0, 0])), np.eye(3))
    for _ in range(20):
        a1, a2 = rng.normal(size=3), rng.normal(size=3)
        R = PR.gram_schmidt(a1, a2)
        assert np.allclose(R.T @ R, np.eye(3), atol=1e-13)
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-12)
        Q = datagen.random_rotation(rng, rng.uniform(0, np.pi))
        assert np.allclose(PR.gram_schmidt(Q @ a1, Q @ a2), Q @ R, atol=1e-12)
        assert np.allclose(PR.gram_schmidt(3.7 * a1, a2 + 2.1 * a1), R, atol=1e-12)
        # the first column is a1's direction, the second lies in span(a1, a2)
        assert np.allclose(R[:, 0], a1 / np.linalg.norm(a1))
        assert abs(np.cross(a1, a2) @ R[:, 1]) < 1e-12


def _torch_forward(theta, xs, ys):
    p = {k: torch.from_numpy(v) for k, v in PR.unpack(theta).items()}
    F = torch.nn.functional

    def enc(x):
        h = F.relu(F.linear(torch.from_numpy(x), p["W1"], p["b1"]))
        h = F.relu(F.linear(h, p["W2"], p["b2"]))
        h = F.relu(F.linear(h, p["W3"], p["b3"]))
        return torch.amax(h, dim=0)

    z = torch.cat([enc(xs), enc(ys)])
    h4 = F.relu(F.linear(z, p["W4"], p["b4"]))
    return F.linear(h4, p["W5"], p["b5"]).numpy()


def test_forward_against_torch():
    rng = np.random.default_rng(1)
    theta = PR.init_params(rng)
    theta += rng.normal(0, 0.02, theta.shape)  # break the near-identity head
    for P in (1, 7, 64):
        xs, ys = rng.normal(size=(P, 3)), rng.normal(size=(P, 3))
        pp = PR.forward_pair(PR.unpack(theta), xs, ys)
        np.testing.assert_allclose(pp.o, _torch_forward(theta, xs, ys), rtol=1e-12, atol=1e-13)
        # source features first: swapping the clouds changes the output
        swapped = PR.forward_pair(PR.unpack(theta), ys, xs)
        assert np.abs(swapped.o - pp.o).max() > 1e-6


def test_initial_prediction_is_near_identity():
    rng = np.random.default_rng(2)
    theta = PR.init_params(rng)
    xs, ys = rng.normal(size=(50, 3)), rng.normal(size=(50, 3))
    pp = PR.forward_pair(PR.unpack(theta), xs, ys)
    assert np.abs(pp.R - np.eye(3)).max() < 0.5


def _small_problem(seed, B=2, P=6):
    rng = np.random.default_rng(seed)
    theta = PR.init_params(rng) + rng.normal(0, 0.05, PR.NPARAM)
    X = rng.normal(size=(B, P, 3))
    Y = rng.normal(size=(B, P, 3))
    R_l = np.stack([datagen.random_rotation(rng, rng.uniform(0, 3)) for _ in range(B)])
    t_l = rng.normal(size=(B, 3)) * 0.3
    return theta, X, Y, R_l, t_l


def test_gradients_against_finite_differences():
    theta, X, Y, R_l, t_l = _small_problem(3)
    _, g, passes = PR.batch_loss_and_grad(theta, X, Y, R_l, t_l)
    # keep the pooling points fixed (the loss is piecewise smooth; the
    # argmax does not move for a step of 1e-6 away from ties)
    am = [(pp.src.idx, pp.tgt.idx) for pp in passes]
    rng = np.random.default_rng(4)
    o = 0
    checked = 0
    for name, shape in PR.SIZES:
        n = int(np.prod(shape))
        for j in rng.choice(n, size=min(n, 12), replace=False):
            i = o + j
            h = 1e-6
            tp, tm = theta.copy(), theta.copy()
            tp[i] += h
            tm[i] -= h
            lp = PR.batch_loss_and_grad(tp, X, Y, R_l, t_l, argmax=am)[0]
            lm = PR.batch_loss_and_grad(tm, X, Y, R_l, t_l, argmax=am)[0]
            fd = (lp - lm) / (2 * h)
            assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-8), (name, j, g[i], fd)
            checked += 1
        o += n
    assert checked > 80


def test_loss_is_least_squares_on_the_6d_outputs():
    """The loss is 0 exactly when the outputs are the label's first two
    columns and translation, and a half-turn label still has a gradient."""
    rng = np.random.default_rng(5)
    theta, X, Y, R_l, t_l = _small_problem(11, B=1)
    pp = PR.forward_pair(PR.unpack(theta), X[0], Y[0])
    R = datagen.random_rotation(rng, 2.0)
    assert PR.pair_loss(pp, R, t_l[0]) == pytest.approx(
        np.sum((pp.o[:3] - R[:, 0]) ** 2) + np.sum((pp.o[3:6] - R[:, 1]) ** 2)
        + np.sum((pp.o[6:] - t_l[0]) ** 2))
    # outputs equal to the target: zero loss
    R0 = PR.gram_schmidt(pp.o[:3], pp.o[3:6])
    n1 = np.linalg.norm(pp.o[:3])
    if abs(n1 - 1.0) < 1e-12 and abs(R0[:, 1] @ pp.o[3:6] - 1.0) < 1e-12:
        assert PR.pair_loss(pp, R0, pp.o[6:]) == pytest.approx(0.0, abs=1e-20)
    # the prediction's own rotation turned by a half turn about its first
    # axis: the second output vector is still pulled towards the label
    flip = R0 @ np.diag([1.0, -1.0, -1.0])
    _, g, _ = PR.batch_loss_and_grad(theta, X, Y, flip[None], t_l)
    assert np.abs(PR.unpack(g)["b5"][3:6]).max() > 0.1


def test_inactive_channels_have_no_gradient():
    """A channel whose every point is inactive pools to 0 and passes no
    gradient to W3's row."""
    theta, X, Y, R_l, t_l = _small_problem(6)
    prm = PR.unpack(theta)
    prm["b3"][5] = -1e3  # channel 5 inactive everywhere
    theta = PR.pack(prm)
    _, g, passes = PR.batch_loss_and_grad(theta, X, Y, R_l, t_l)
    assert all(pp.src.f[5] == 0.0 and pp.tgt.f[5] == 0.0 for pp in passes)
    gW3 = PR.unpack(g)["W3"]
    assert np.all(gW3[5] == 0.0) and PR.unpack(g)["b3"][5] == 0.0


def test_adam_closed_form():
    rng = np.random.default_rng(7)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    z = np.zeros(50)
    lr = 1e-3
    t1, m1, v1 = PR.adam_step(theta, g, z, z, 1, lr)
    # bias-corrected first step: m^ = g, v^ = g^2
    np.testing.assert_allclose(t1, theta - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    g2 = rng.normal(size=50)
    t2, _, _ = PR.adam_step(t1, g2, m1, v1, 2, lr)
    m = 0.9 * 0.1 * g + 0.1 * g2
    v = 0.999 * 0.001 * g * g + 0.001 * g2 * g2
    mh, vh = m / (1 - 0.81), v / (1 - 0.999 ** 2)
    np.testing.assert_allclose(t2, t1 - lr * mh / (np.sqrt(vh) + 1e-8), rtol=0, atol=1e-15)


def test_sampling_and_normalisation_round_trip():
    assert list(PR.sample_indices(10, 5)) == [1, 3, 5, 7, 9]
    assert list(PR.sample_indices(3, 6)) == [0, 0, 1, 1, 2, 2]
    assert list(PR.sample_indices(7, 7)) == list(range(7))
    # one sample: no spread, unit scale and frame, both inputs at the origin
    xs1, ys1, (_, _, s1, FX1, FY1) = PR.normalise(np.ones((5, 3)), np.arange(12.0).reshape(4, 3), 1)
    assert s1 == 1.0 and not xs1.any() and not ys1.any()
    assert np.array_equal(FX1, np.eye(3)) and np.array_equal(FY1, np.eye(3))
    rng = np.random.default_rng(8)
    p = datagen.range_scanner_pair(trial=2, M=900, N=700)
    Q = datagen.random_rotation(rng, 2.0)
    xs, ys, norm = PR.normalise(p.X, p.Y, 256, Q)
    assert np.allclose(xs.mean(0), 0, atol=1e-12) and np.allclose(ys.mean(0), 0, atol=1e-12)
    assert np.mean(np.sum(ys ** 2, axis=1)) == pytest.approx(1.0)
    # the pose mapping x' = Q x onto y: R_gt Q^T, t_gt
    R = p.R_gt @ Q.T
    Rc, tc = PR.label_normalised(R, p.t_gt, norm)
    R2, t2 = PR.pose_from_prediction(Rc, tc, norm)
    assert np.allclose(R2, R) and np.allclose(t2, p.t_gt, atol=1e-12)
    # in these units the label maps the source's inputs onto the inputs of
    # the image of the same points
    mx, my, s, FX, FY = norm
    raw = np.asarray(p.X, np.float64)[PR.sample_indices(700, 256)] @ Q.T
    img = (((raw @ R.T + p.t_gt) - my) @ FY) / s
    np.testing.assert_allclose(xs @ Rc.T + tc, img, atol=1e-12)


def test_principal_frame():
    """Eigenvectors of the covariance in decreasing order of eigenvalue,
    right-handed, third moments along e0, e1 non-negative; rotating the
    points rotates the frame and leaves the inputs unchanged."""
    rng = np.random.default_rng(9)
    c = rng.normal(size=(300, 3)) * [3.0, 1.5, 0.5] + rng.exponential(size=(300, 3)) * 0.3
    c -= c.mean(0)
    F = PR.principal_frame(c)
    assert np.allclose(F.T @ F, np.eye(3), atol=1e-12) and np.linalg.det(F) == pytest.approx(1.0)
    C = c.T @ c / len(c)
    lam = np.diag(F.T @ C @ F)
    assert np.all(np.diff(lam) < 0)
    np.testing.assert_allclose(F.T @ C @ F, np.diag(lam), atol=1e-12 * lam[0])
    assert np.sum((c @ F[:, 0]) ** 3) >= 0 and np.sum((c @ F[:, 1]) ** 3) >= 0
    Q = datagen.random_rotation(rng, 2.5)
    np.testing.assert_allclose(PR.principal_frame(c @ Q.T), Q @ F, atol=1e-10)
    p = datagen.range_scanner_pair(trial=3, M=800, N=600)
    xs, ys, _ = PR.normalise(p.X, p.Y, 200)
    xq, yq, _ = PR.normalise(p.X, p.Y, 200, Q)
    np.testing.assert_allclose(xq, xs, atol=1e-10)
    np.testing.assert_allclose(yq, ys, atol=0)
