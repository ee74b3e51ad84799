"""Registrations whose EM loop is replayed from a HIP graph recording
(LSGCPD_GRAPH) against the same registrations launched kernel by kernel.

Bar: bitwise equality (the same kernels run in the same order on the same
data).  The recording is replayed several times with eager GPU work and
synchronisations in between, for new clouds of the same sizes (the clouds are
reached through tables uploaded per call), re-recorded for other sizes, and
used by batches and by the tolerance stop."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2103_15039_amd")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _same(a, b):
    assert a.iters == b.iters and a.converged == b.converged
    assert np.array_equal(a.R, b.R) and np.array_equal(a.t, b.t)
    assert a.sigma2 == b.sigma2
    assert np.array_equal(a.nll, b.nll)


def test_graph_replays_equal_eager():
    rng = datagen.rng_for(13, 0)
    p1 = datagen.scene_pair(rng, 1500, 1200, max_angle_deg=25.0)
    p3 = datagen.scene_pair(rng, 1500, 1200, max_angle_deg=25.0)   # same sizes as p1
    p2 = datagen.scene_pair(rng, 900, 2100, max_angle_deg=25.0)
    kw = dict(k=10, max_iter=30)
    clouds = [(dev(p.X), dev(p.Y)) for p in (p1, p2, p3)]
    eager = [L.register(X, Y, **kw) for X, Y in clouds]
    for rep in range(3):
        for (X, Y), e in zip(clouds, eager):
            g = L.register(X, Y, graph=True, **kw)
            _same(g, e)
            # eager work on the same stream between replays
            junk = (X * 2.0).sum() + Y.mean()
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
    # new tensors (other addresses) with the same sizes replay the recording
    X1b, Y1b = clouds[0][0].clone(), clouds[0][1].clone()
    _same(L.register(X1b, Y1b, graph=True, **kw), eager[0])


def test_graph_tolerance_stop_and_batch():
    rng = datagen.rng_for(13, 1)
    p = datagen.scene_pair(rng, 2000, 1800, max_angle_deg=20.0)
    X, Y = dev(p.X), dev(p.Y)
    kw = dict(k=10, max_iter=80, tol=1e-7)
    e = L.register(X, Y, **kw)
    assert e.converged
    for _ in range(2):
        _same(L.register(X, Y, graph=True, **kw), e)
    pairs = [datagen.scene_pair(rng, M, N, max_angle_deg=25.0)
             for M, N in [(700, 900), (2500, 400), (60, 50)]]
    args = [(dev(q.X), dev(q.Y)) for q in pairs]
    be = L.register_batch(args, k=8, max_iter=25)
    for _ in range(2):
        bg = L.register_batch(args, k=8, max_iter=25, graph=True)
        for a, b in zip(bg, be):
            _same(a, b)
        torch.cuda.synchronize()
