"""The BF16 matrix-core exponent (LSGCPD_BF16_CROSS) against the FP64 oracle.

The path evaluates c d_mn as a product of lifted quadratic features (the
bilinear structure of Eq. 10), each split into BF16 high and low parts, about
the box centre of each half of 64 sources, with FP32 sums, and accumulates
e [1, f_m] as a second BF16 product.  It is an approximation with a stated
error, not a parity path:
  * per pair, |dz| <= 4.96e-5 (1 + alpha_m) (|u| + |v|)^2, with u and v the
    source and the target in scaled units (sqrt(c) times the coordinates)
    about the centre of the source's half box; the accumulation adds at most
    2^-15 relative to each term;
  * an E step takes the path only while that bound is below 1/32 for every
    pair within scaled distance 2 of every source half; otherwise the FP64
    kernel runs and the parity bar holds as without the flag.
The tests check the per-pair bound with one target (the per-source sum is
then the pair's exponential), per-source sums and statistics with many
targets, the switch back to FP64 at small sigma^2, and whole registrations,
whose final poses (the late, small-sigma^2 E steps run in FP64) must meet the
registration bar (1e-3 deg, 1e-5 of the box diagonal).
"""
import numpy as np
import pytest

import datagen
from oracle import lsgcpd_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
L = pytest.importorskip("paper_2103_15039_amd")

KAPPA = 3.0 / 65536.0 + 64.0 / 16777216.0
LOG2E = 1.4426950408889634


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _case(M, N, seed, amax=30.0):
    p = datagen.range_scanner_pair(trial=seed, M=M, N=N)
    rng = np.random.default_rng(seed)
    n = datagen.random_unit_normals(rng, M).astype(np.float32)
    a = rng.uniform(0.0, amax, M).astype(np.float32)
    R = datagen.random_rotation(rng, 0.3) @ p.R_gt
    t = p.t_gt + rng.uniform(-0.05, 0.05, 3)
    return p.X, p.Y, n, a, R, t


def _pair_bound(X, Y, a, R, t, s2):
    """The stated |dz| bound of every (target, source) pair: the sources'
    half boxes of 64 in the caller's order, scaled coordinates."""
    sc = np.sqrt(LOG2E / (2.0 * s2))
    S = (X.astype(np.float64) @ R.T + t) * sc
    V = Y.astype(np.float64) * sc
    N = len(S)
    bound = np.empty((len(Y), N))
    for h0 in range(0, N, 64):
        Sh = S[h0:h0 + 64]
        o = 0.5 * (Sh.min(0) + Sh.max(0))
        u = np.linalg.norm(Sh - o, axis=1)
        v = np.linalg.norm(V - o, axis=1)
        bound[:, h0:h0 + 64] = KAPPA * (1.0 + a.astype(np.float64))[:, None] * (u[None, :] + v[:, None]) ** 2
    return bound


def test_per_pair_exponent_within_bound():
    """One target: the per-source sum T0_n = sum_m e_mn is the pair's own
    exponential, so its error against the oracle is the pair's error."""
    X, Y, n, a, R, t = _case(1, 3000, seed=1, amax=25.0)
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    for s2 in (0.6, 1.0):
        g = L.estep(dev(X), dev(Y), dev(n), dev(a), R, t, s2, w0=0.1, colstats=True, bf16=True)
        assert g.bf16_cross
        es = O.estep(Xd, Yd, n.astype(np.float64), a.astype(np.float64), R, t, s2, w0=0.1)
        rho = (1.0 - 0.1) / 0.1
        e_ref = es.Ksum / rho
        e_gpu = g.colstats.cpu().numpy()[:, 0]
        dz = np.abs(np.log2(e_gpu / e_ref))
        b = _pair_bound(X, Y, a, R, t, s2)[0]
        # accumulation: e_hi + e_lo is e to 2^-16; float32 exp2 and rounding of z
        slack = 2.0 ** -15 / np.log(2.0) + 1e-6 * (1.0 + np.abs(np.log2(e_ref)))
        worst = np.argmax(dz - b - slack)
        assert np.all(dz <= b + slack), (s2, worst, dz[worst], b[worst])
        # typical errors are far inside the worst-case bound
        assert np.median(dz) < 1e-3


@pytest.mark.parametrize("M,N,s2", [(700, 900, 1.0), (2000, 2000, 2.0)])
def test_estep_sums_and_statistics(M, N, s2):
    X, Y, n, a, R, t = _case(M, N, seed=M + 3)
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    nd, ad = n.astype(np.float64), a.astype(np.float64)
    g = L.estep(dev(X), dev(Y), dev(n), dev(a), R, t, s2, w0=0.1, colstats=True, bf16=True)
    assert g.bf16_cross
    es = O.estep(Xd, Yd, nd, ad, R, t, s2, w0=0.1)
    rho = 9.0
    cs = g.colstats.cpu().numpy()
    b = _pair_bound(X, Y, a, R, t, s2)
    # per source, the sum's relative error is at most the largest of its
    # terms' (each e_mn within 2^(bound) of the exact value)
    rel = np.abs(cs[:, 0] * rho / es.Ksum - 1.0)
    allowed = np.expm1(np.log(2.0) * b.max(axis=0)) + 2.0 ** -15
    assert np.all(rel <= allowed)
    cols = O.columns(es.P, Xd, Yd, nd, ad, R, t)
    ref = O.lifted_stats(cols, Xd, O.nll_terms(es, None, 0.1))
    # the statistics inherit the relative error of the weights: stated, and
    # checked against the largest per-pair bound of the E step
    scale = np.abs(ref) + 1e-9 * np.abs(ref).max()
    err = np.abs(g.stats - ref) / scale
    assert err[:83].max() <= np.expm1(np.log(2.0) * b.max()) + 2.0 ** -14
    assert g.nll == pytest.approx(es.nll, rel=1e-3)


def test_small_sigma2_runs_fp64_kernel():
    """At small sigma^2 the bound fails and the E step is the FP64 one: the
    parity bar holds exactly as without the flag."""
    X, Y, n, a, R, t = _case(800, 700, seed=9)
    s2 = 2e-3
    g = L.estep(dev(X), dev(Y), dev(n), dev(a), R, t, s2, w0=0.1, bf16=True, dump_P=True)
    assert not g.bf16_cross
    ref = L.estep(dev(X), dev(Y), dev(n), dev(a), R, t, s2, w0=0.1, dump_P=True)
    np.testing.assert_array_equal(g.stats, ref.stats)
    es = O.estep(X.astype(np.float64), Y.astype(np.float64), n.astype(np.float64),
                 a.astype(np.float64), R, t, s2, w0=0.1)
    P = g.P.double().cpu().numpy()
    assert np.all(np.abs(P - es.P) <= 1e-5 * es.P + 1e-10)


@pytest.mark.parametrize("workload", ["range_scanner", "rgbd"])
def test_registration_meets_bar(workload):
    """Early E steps on the matrix cores, late ones in FP64: the final pose
    against the all-FP64 oracle registration."""
    if workload == "range_scanner":
        p = datagen.range_scanner_pair(trial=0)
        k, iters = 10, 50
    else:
        p = datagen.rgbd_pair(0)
        k, iters = 20, 50
    r = L.register(dev(p.X), dev(p.Y), k=k, max_iter=iters, bf16=True)
    assert r.bf16_steps >= 1
    base = L.register(dev(p.X), dev(p.Y), k=k, max_iter=iters)
    assert base.bf16_steps == 0
    diag = O.bbox_diag(p.Y.astype(np.float64))
    assert O.rotation_error_deg(r.R, base.R) <= 1e-3
    assert O.translation_error(r.t, base.t) <= 1e-5 * diag
    if workload == "range_scanner":
        o = O.register(p.X, p.Y, k=k, max_iter=iters)
        assert O.rotation_error_deg(r.R, o.R) <= 1e-3
        assert O.translation_error(r.t, o.t) <= 1e-5 * diag


def test_flag_combinations_rejected():
    X, Y, n, a, R, t = _case(100, 100, seed=4)
    for backend in ("dense", "lds", "mfma"):
        with pytest.raises(L.LsgcpdError) as e:
            L.estep(dev(X), dev(Y), dev(n), dev(a), R, t, 1.0, bf16=True, backend=backend)
        assert e.value.status == L.E_INVALID
