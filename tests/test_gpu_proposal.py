"""GPU parity of the learned initial-pose proposal against its FP64 oracle
(oracle/proposal_ref.py), through the C ABI:
  * encoder inputs (sampling, rotation, centring, principal-axis frames,
    scale): float32 rounding of the oracle's values, frames to 1e-9;
  * forward poses, with ragged point counts (not multiples of the 64-point
    blocks) and a single point: rotation entries within 2e-4, translations
    within 2e-4 of the target scale (FP32 products of 41k MACs per point);
  * one training step: the loss per pair (relative 1e-4), the pooled points
    (where two points' activations are within FP32 rounding the GPU may pick
    either: its choice must be a maximum of the oracle's activations to 1e-5,
    and the oracle's gradient is then taken at the GPU's choice), the
    gradient (every parameter within 1e-3 of the largest gradient of its
    layer), and the Adam update (within 1e-6 absolute, the update being lr
    times a ratio of FP32 moments);
  * batches built from stored inputs by index equal the same pairs built
    directly (bitwise);
  * the fallback of lsgcpd_register_proposed keeps the lowest-NLL run of
    the frame-aligned starts it ran.
"""
import numpy as np
import pytest

import datagen
from oracle import proposal_ref as PR

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2103_15039_amd")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _pairs(n, seed, nmin=150, nmax=900):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        M, N = (int(v) for v in rng.integers(nmin, nmax, 2))
        out.append(datagen.proposal_pair(rng, M, N))
    return out


def _theta(seed):
    rng = np.random.default_rng(seed)
    th = PR.init_params(rng)
    return th + rng.normal(0, 0.02, th.shape)


def _norm_tuple(row):
    return (row[0:3], row[3:6], row[6], row[7:16].reshape(3, 3), row[16:25].reshape(3, 3))


def test_inputs_match_oracle():
    ps = _pairs(3, 1)
    rng = np.random.default_rng(2)
    Q = np.stack([datagen.uniform_rotation(rng) for _ in ps])
    for P, q in ((256, None), (100, Q), (1000, Q)):
        Xn, Yn, norm = L.proposal_inputs([(dev(p.X), dev(p.Y)) for p in ps], P, q)
        Xn, Yn, norm = Xn.cpu().numpy(), Yn.cpu().numpy(), norm.cpu().numpy()
        for i, p in enumerate(ps):
            xs, ys, (mx, my, s, FX, FY) = PR.normalise(p.X, p.Y, P, None if q is None else q[i])
            np.testing.assert_allclose(Xn[i], xs, rtol=0, atol=2e-6 * max(1.0, np.abs(xs).max()))
            np.testing.assert_allclose(Yn[i], ys, rtol=0, atol=2e-6 * max(1.0, np.abs(ys).max()))
            g = _norm_tuple(norm[i])
            np.testing.assert_allclose(g[0], mx, rtol=1e-12, atol=1e-14)
            np.testing.assert_allclose(g[1], my, rtol=1e-12, atol=1e-14)
            assert g[2] == pytest.approx(s, rel=1e-12)
            np.testing.assert_allclose(g[3], FX, atol=1e-9)
            np.testing.assert_allclose(g[4], FY, atol=1e-9)


@pytest.mark.parametrize("P", [1, 37, 200, 512])
def test_forward_matches_oracle(P):
    ps = _pairs(4, 10 + P)
    theta = _theta(P)
    Xn, Yn, norm = L.proposal_inputs([(dev(p.X), dev(p.Y)) for p in ps], P)
    pose = L.proposal_forward(dev(theta), Xn, Yn, norm).cpu().numpy()
    prm = PR.unpack(theta.astype(np.float32).astype(np.float64))
    for i, p in enumerate(ps):
        xs, ys, nm = PR.normalise(p.X, p.Y, P)
        pp = PR.forward_pair(prm, Xn[i].cpu().numpy().astype(np.float64),
                             Yn[i].cpu().numpy().astype(np.float64))
        R, t = PR.pose_from_prediction(pp.R, pp.t, nm)
        np.testing.assert_allclose(pose[i, :9].reshape(3, 3), R, rtol=0, atol=2e-4)
        np.testing.assert_allclose(pose[i, 9:], t, rtol=0, atol=2e-4 * nm[2])


def _layer_check(g_gpu, g_ref):
    o = 0
    for name, shape in PR.SIZES:
        n = int(np.prod(shape))
        a, b = g_gpu[o:o + n], g_ref[o:o + n]
        scale = max(np.abs(b).max(), 1e-12)
        worst = np.argmax(np.abs(a - b))
        assert np.abs(a - b).max() <= 1e-3 * scale, (name, worst, a[worst], b[worst], scale)
        o += n


@pytest.mark.parametrize("B,P", [(3, 130), (5, 64)])
def test_train_step_matches_oracle(B, P):
    ps = _pairs(B, 20 + B)
    theta = _theta(40 + B)
    Xn, Yn, norm = L.proposal_inputs([(dev(p.X), dev(p.Y)) for p in ps], P)
    # labels: the ground-truth pose from the source to the target
    label = np.stack([np.concatenate([p.R_gt.ravel(), p.t_gt]) for p in ps])
    th = dev(theta)
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    lr = 1e-3
    loss, am, g = L.proposal_train_step(th, m, v, 1, lr, Xn, Yn, norm, label,
                                        want_argmax=True, want_grad=True)
    loss, am, g = loss.cpu().numpy(), am.cpu().numpy(), g.cpu().numpy().astype(np.float64)
    th32 = theta.astype(np.float32).astype(np.float64)
    prm = PR.unpack(th32)
    Xin = Xn.cpu().numpy().astype(np.float64)
    Yin = Yn.cpu().numpy().astype(np.float64)
    nrm = norm.cpu().numpy()
    Rl, tl = [], []
    for i in range(B):
        R, t = PR.label_normalised(label[i, :9].reshape(3, 3), label[i, 9:], _norm_tuple(nrm[i]))
        Rl.append(R)
        tl.append(t)
    # the GPU's pooled points must be maxima of the oracle's activations
    for i in range(B):
        for side, x in ((0, Xin[i]), (1, Yin[i])):
            cp = PR.encode(prm, x)
            h3 = np.maximum(cp.a3, 0.0)
            picked = h3[am[i, side], np.arange(256)]
            assert np.all(picked >= h3.max(axis=0) - 1e-5 * (1.0 + h3.max(axis=0)))
    ref_loss, g_ref, passes = PR.batch_loss_and_grad(th32, Xin, Yin, np.stack(Rl), np.stack(tl),
                                                     argmax=[(am[i, 0], am[i, 1]) for i in range(B)])
    per_pair = [PR.pair_loss(pp, Rl[i], tl[i]) for i, pp in enumerate(passes)]
    np.testing.assert_allclose(loss, per_pair, rtol=1e-4)
    _layer_check(g, g_ref)
    # Adam, first step, from the GPU's own gradient
    t1, _, _ = PR.adam_step(th32, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    np.testing.assert_allclose(th.cpu().numpy(), t1, rtol=0, atol=1e-6)


def test_indexed_batch_equals_direct_batch():
    ps = _pairs(4, 50)
    index = np.array([2, 0, 3, 3, 1, 2], np.int32)
    P = 96
    theta = _theta(52)
    Xn, Yn, norm = L.proposal_inputs([(dev(p.X), dev(p.Y)) for p in ps], P)
    Xd, Yd, nd = L.proposal_inputs([(dev(ps[j].X), dev(ps[j].Y)) for j in index], P)
    label = np.stack([np.concatenate([ps[j].R_gt.ravel(), ps[j].t_gt]) for j in index])
    outs = []
    for args in ((Xn, Yn, norm, index), (Xd, Yd, nd, None)):
        th = dev(theta)
        m, v = torch.zeros_like(th), torch.zeros_like(th)
        loss, _, g = L.proposal_train_step(th, m, v, 1, 1e-3, args[0], args[1], args[2], label,
                                           index=args[3], want_grad=True)
        outs.append((loss.cpu().numpy(), g.cpu().numpy()))
    np.testing.assert_allclose(outs[0][0], outs[1][0], rtol=1e-6)
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


def test_training_reduces_the_loss():
    """200 Adam steps on 64 fixed pairs: the mean loss falls (behaviour, not
    parity)."""
    ps = _pairs(64, 60, nmin=300, nmax=600)
    P = 128
    Xn, Yn, norm = L.proposal_inputs([(dev(p.X), dev(p.Y)) for p in ps], P)
    rng = np.random.default_rng(61)
    th = dev(PR.init_params(rng))
    m, v = torch.zeros_like(th), torch.zeros_like(th)
    labels = np.stack([np.concatenate([p.R_gt.ravel(), p.t_gt]) for p in ps])
    first, last = [], []
    for step in range(1, 201):
        index = rng.integers(0, 64, 32).astype(np.int32)
        loss, _, _ = L.proposal_train_step(th, m, v, step, 1e-3, Xn, Yn, norm, labels[index],
                                           index=index)
        (first if step <= 20 else last if step > 180 else []).append(float(loss.mean()))
    assert np.isfinite(last).all()
    assert np.mean(last) < 0.7 * np.mean(first)


def test_invalid_arguments():
    ps = _pairs(1, 70)
    with pytest.raises(L.LsgcpdError) as e:
        L.proposal_inputs([(dev(ps[0].X), dev(ps[0].Y))], 5000)
    assert e.value.status == L.E_INVALID
    Xn, Yn, norm = L.proposal_inputs([(dev(ps[0].X), dev(ps[0].Y))], 64)
    th = dev(np.zeros(L.PROPOSAL_PARAMS))
    z = torch.zeros_like(th)
    with pytest.raises(L.LsgcpdError) as e:
        L.proposal_train_step(th, z, z.clone(), 0, 1e-3, Xn, Yn, norm, np.zeros((1, 12)))
    assert e.value.status == L.E_INVALID
    with pytest.raises(L.LsgcpdError) as e:   # index beyond the stored pairs
        L.proposal_train_step(th, z, z.clone(), 1, 1e-3, Xn, Yn, norm, np.zeros((1, 12)),
                              index=[1])
    assert e.value.status == L.E_INVALID


def _cube_rotations():
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1.0, -1.0), repeat=3):
            R = np.zeros((3, 3))
            for r in range(3):
                R[r, perm[r]] = signs[r]
            if np.linalg.det(R) > 0:
                out.append(R)
    return out


def test_register_proposed_falls_back_to_frame_starts():
    """With an untrained encoder and sources rotated far from their targets,
    the pairs it does not accept are registered from the frame-aligned
    starts R = F_Y G F_X^T (G: the 24 rotations of the cube), and the run
    kept has the lowest final NLL among the proposal's run and the starts
    that ran: at most the best of the 24 single-pair runs from the same
    starts unless the pair was accepted after the 4 sign changes."""
    rng = np.random.default_rng(80)
    ps = []
    while len(ps) < 4:
        p = datagen.proposal_pair(rng, 600, 500)
        ang = np.degrees(np.arccos(np.clip((np.trace(p.R_gt) - 1) / 2, -1, 1)))
        if ang > 100:
            ps.append(p)
    theta = dev(PR.init_params(np.random.default_rng(81)))
    P = 256
    kw = dict(k=10, max_iter=40)
    res, fb = L.register_proposed([(dev(p.X), dev(p.Y)) for p in ps], theta, P=P, accept=0.05, **kw)
    assert fb.sum() >= 1
    G = _cube_rotations()
    assert len(G) == 24
    signs = [g for g in G if np.count_nonzero(g) == 3 and np.allclose(g, np.diag(np.diag(g)))]
    assert len(signs) == 4
    for i, p in enumerate(ps):
        if not fb[i]:
            continue
        _, _, (mx, my, s, FX, FY) = PR.normalise(p.X, p.Y, P)

        def run(g):
            R = FY @ g @ FX.T
            return L.register(dev(p.X), dev(p.Y), R0=R, t0=my - R @ mx, **kw)
        best4 = min(run(g).nll[-1] for g in signs)
        assert res[i].nll[-1] <= best4 + 1e-6 * abs(best4)
        if np.sqrt(res[i].sigma2) > 0.05 * s:  # not accepted: all 24 starts ran
            best = min(run(g).nll[-1] for g in G)
            assert res[i].nll[-1] <= best + 1e-6 * abs(best)
