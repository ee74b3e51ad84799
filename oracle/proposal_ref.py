"""Plain FP64 reference of the learned initial-pose proposal: a point-set
encoder that predicts the rigid motion between two clouds, used to start
LSG-CPD near the right pose (the method needs a start inside its basin of
convergence: Sec. 1 and Sec. 5 of the paper on sensitivity to
initialisation).

TEST INFRASTRUCTURE ONLY.  This module is the oracle that the GPU proposal
kernels are checked against.  Only the test-suite may import it; the library
never does, and nothing here is shared with the GPU code.

The model (sizes from the project's configuration of the proposal):
  * each cloud, P points normalised as below, goes through a shared per-point
    MLP 3 -> 64 -> 128 -> 256 (ReLU after every layer) and a max-pool over
    its points: one 256-vector per cloud;
  * the source's and the target's vectors, side by side (512), go through
    512 -> 128 (ReLU) -> 9;
  * outputs 0..5 are two 3-vectors turned into a rotation by Gram-Schmidt
    (the continuous 6-D representation of Zhou et al., CVPR 2019), outputs
    6..8 the translation in normalised units.
Parameters are one flat float vector, layer by layer, each W row-major
[out][in] followed by its b:
  W1 64x3, b1 64, W2 128x64, b2 128, W3 256x128, b3 256, W4 128x512, b4 128,
  W5 9x128, b5 9   (108,425 values).
Input normalisation (one cloud pair, optional rotation Q of the source):
  * P points of a cloud of N are taken at indices floor((2k + 1) N / (2P)),
    k = 0 .. P-1 (evenly spaced in the cloud's order; repeats when N < P);
  * x' = Q x; mu_X = mean of the sampled x', mu_Y = mean of the sampled y;
    s = root-mean-square distance of the sampled y from mu_Y;
  * inputs (x' - mu_X) / s and (y - mu_Y) / s (s = 1 when the target's
    samples are all one point, e.g. P = 1).
A pose (R, t) mapping x' onto y reads, in normalised units, R and
t^ = (R mu_X + t - mu_Y) / s; a prediction (R^, t^) maps back to
t = mu_Y + s t^ - R^ mu_X.
Loss of a pair: |R^ - R_label|_F^2 + |t^ - t^_label|^2; of a batch: the mean.
Optimiser: Adam (Kingma and Ba, ICLR 2015) with bias correction,
beta1 = 0.9, beta2 = 0.999, eps = 1e-8.

Max-pool ties go to the lower point index.  Where a channel's largest
activation is 0 (every point inactive), its gradient is 0.

Parity status: pinned by tests/test_oracle_proposal.py -- Gram-Schmidt against
its closed-form properties, the forward pass against an independent float64
implementation in torch, every gradient against central finite differences,
Adam against its published update in closed form, and the normalisation and
pose mapping by round trips.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SIZES = [("W1", (64, 3)), ("b1", (64,)), ("W2", (128, 64)), ("b2", (128,)),
         ("W3", (256, 128)), ("b3", (256,)), ("W4", (128, 512)), ("b4", (128,)),
         ("W5", (9, 128)), ("b5", (9,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


def unpack(theta):
    """Views of the flat parameter vector, by name."""
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], np.float64).ravel() for name, _ in SIZES])


def sample_indices(N, P):
    """Evenly spaced indices floor((2k + 1) N / (2P)), integer arithmetic."""
    k = np.arange(P, dtype=np.int64)
    return ((2 * k + 1) * int(N)) // (2 * int(P))


def normalise(X, Y, P, Q=None):
    """Encoder inputs of one pair and the normalisation (mu_X, mu_Y, s)."""
    xs = np.asarray(X, np.float64)[sample_indices(len(X), P)]
    ys = np.asarray(Y, np.float64)[sample_indices(len(Y), P)]
    if Q is not None:
        xs = xs @ np.asarray(Q, np.float64).T
    mx, my = xs.mean(axis=0), ys.mean(axis=0)
    s = np.sqrt(np.mean(np.sum((ys - my) ** 2, axis=1)))
    if not s > 0.0:
        s = 1.0  # the target's samples are one point: no scale to take
    return (xs - mx) / s, (ys - my) / s, (mx, my, s)


def label_normalised(R, t, norm):
    """(R, t^) of a pose mapping x' onto y, in the normalised units of norm."""
    mx, my, s = norm
    return np.asarray(R, np.float64), (np.asarray(R) @ mx + np.asarray(t) - my) / s


def pose_from_prediction(R_hat, t_hat, norm):
    """World pose of a normalised prediction."""
    mx, my, s = norm
    return np.asarray(R_hat, np.float64), my + s * np.asarray(t_hat) - R_hat @ mx


def gram_schmidt(a1, a2):
    """Rotation whose columns are a1 normalised, the part of a2 orthogonal to
    it normalised, and their cross product."""
    b1 = a1 / np.linalg.norm(a1)
    u2 = a2 - (b1 @ a2) * b1
    b2 = u2 / np.linalg.norm(u2)
    b3 = np.cross(b1, b2)
    return np.stack([b1, b2, b3], axis=1)


def gram_schmidt_backward(a1, a2, dR):
    """Gradients of sum(dR * R) with respect to a1 and a2."""
    n1 = np.linalg.norm(a1)
    b1 = a1 / n1
    c = b1 @ a2
    u2 = a2 - c * b1
    n2 = np.linalg.norm(u2)
    b2 = u2 / n2
    g1, g2, g3 = dR[:, 0], dR[:, 1], dR[:, 2]
    # b3 = b1 x b2: d<g3, b1 x b2> = <b2 x g3, db1> + <g3 x b1, db2>
    gb1 = g1 + np.cross(b2, g3)
    gb2 = g2 + np.cross(g3, b1)
    # b2 = u2 / |u2|
    gu2 = (gb2 - (gb2 @ b2) * b2) / n2
    # u2 = a2 - (b1 . a2) b1
    ga2 = gu2 - (gu2 @ b1) * b1
    gb1 = gb1 - (gu2 @ b1) * a2 - c * gu2
    # b1 = a1 / |a1|
    ga1 = (gb1 - (gb1 @ b1) * b1) / n1
    return ga1, ga2


@dataclass
class CloudPass:
    x: np.ndarray      # (P, 3) inputs
    h1: np.ndarray     # (P, 64)
    h2: np.ndarray     # (P, 128)
    a3: np.ndarray     # (P, 256) pre-activation of layer 3
    f: np.ndarray      # (256,) pooled
    idx: np.ndarray    # (256,) argmax point of each channel


def encode(prm, x, argmax=None):
    """Per-point MLP and max-pool of one cloud.  argmax: optional forced
    argmax points (must be valid maxima; used to compare tie-breaking)."""
    h1 = np.maximum(x @ prm["W1"].T + prm["b1"], 0.0)
    h2 = np.maximum(h1 @ prm["W2"].T + prm["b2"], 0.0)
    a3 = h2 @ prm["W3"].T + prm["b3"]
    h3 = np.maximum(a3, 0.0)
    idx = np.argmax(h3, axis=0) if argmax is None else np.asarray(argmax, np.int64)
    f = h3[idx, np.arange(h3.shape[1])]
    return CloudPass(x=x, h1=h1, h2=h2, a3=a3, f=f, idx=idx)


@dataclass
class PairPass:
    src: CloudPass
    tgt: CloudPass
    z: np.ndarray      # (512,)
    h4: np.ndarray     # (128,)
    o: np.ndarray      # (9,)
    R: np.ndarray      # (3, 3)
    t: np.ndarray      # (3,) normalised


def forward_pair(prm, xs, ys, argmax_src=None, argmax_tgt=None):
    a = encode(prm, xs, argmax_src)
    b = encode(prm, ys, argmax_tgt)
    z = np.concatenate([a.f, b.f])
    h4 = np.maximum(prm["W4"] @ z + prm["b4"], 0.0)
    o = prm["W5"] @ h4 + prm["b5"]
    R = gram_schmidt(o[0:3], o[3:6])
    return PairPass(src=a, tgt=b, z=z, h4=h4, o=o, R=R, t=o[6:9].copy())


def pair_loss(pp, R_l, t_l):
    return float(np.sum((pp.R - R_l) ** 2) + np.sum((pp.t - t_l) ** 2))


def _encode_backward(prm, cp, gf, grads):
    """Gradients of <gf, f> through the max-pool and the per-point MLP."""
    ga3 = np.zeros_like(cp.a3)
    live = cp.f > 0.0                       # ReLU active at the argmax
    ch = np.nonzero(live)[0]
    ga3[cp.idx[ch], ch] += gf[ch]
    grads["W3"] += ga3.T @ cp.h2
    grads["b3"] += ga3.sum(axis=0)
    gh2 = ga3 @ prm["W3"]
    ga2 = gh2 * (cp.h2 > 0.0)
    grads["W2"] += ga2.T @ cp.h1
    grads["b2"] += ga2.sum(axis=0)
    gh1 = ga2 @ prm["W2"]
    ga1 = gh1 * (cp.h1 > 0.0)
    grads["W1"] += ga1.T @ cp.x
    grads["b1"] += ga1.sum(axis=0)


def batch_loss_and_grad(theta, X_in, Y_in, R_l, t_l, argmax=None):
    """Mean loss over a batch and its gradient (flat).  X_in, Y_in: (B, P, 3)
    normalised inputs; R_l (B, 3, 3), t_l (B, 3) normalised labels; argmax:
    optional (B, 2, 256) forced pooling points."""
    prm = unpack(theta)
    B = len(X_in)
    grads = {name: np.zeros(shape) for name, shape in SIZES}
    total = 0.0
    passes = []
    for i in range(B):
        am = (None, None) if argmax is None else (argmax[i][0], argmax[i][1])
        pp = forward_pair(prm, np.asarray(X_in[i], np.float64), np.asarray(Y_in[i], np.float64),
                          am[0], am[1])
        passes.append(pp)
        total += pair_loss(pp, R_l[i], t_l[i])
        dR = 2.0 * (pp.R - R_l[i]) / B
        dt = 2.0 * (pp.t - t_l[i]) / B
        ga1, ga2 = gram_schmidt_backward(pp.o[0:3], pp.o[3:6], dR)
        go = np.concatenate([ga1, ga2, dt])
        grads["W5"] += np.outer(go, pp.h4)
        grads["b5"] += go
        gh4 = prm["W5"].T @ go
        ga4 = gh4 * (pp.h4 > 0.0)
        grads["W4"] += np.outer(ga4, pp.z)
        grads["b4"] += ga4
        gz = prm["W4"].T @ ga4
        _encode_backward(prm, pp.src, gz[:256], grads)
        _encode_backward(prm, pp.tgt, gz[256:], grads)
    return total / B, pack(grads), passes


def adam_step(theta, grad, m, v, step, lr):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = BETA1 * m + (1.0 - BETA1) * grad
    v = BETA2 * v + (1.0 - BETA2) * grad * grad
    mh = m / (1.0 - BETA1 ** step)
    vh = v / (1.0 - BETA2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + EPS), m, v


def init_params(rng):
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases; the last
    layer scaled by 0.1 and its bias set so that the initial prediction is
    near the identity rotation (a1 = e_x, a2 = e_y) with zero translation."""
    parts = {}
    for name, shape in SIZES:
        if name.startswith("W"):
            bound = np.sqrt(6.0 / shape[1])
            parts[name] = rng.uniform(-bound, bound, shape)
        else:
            parts[name] = np.zeros(shape)
    parts["W5"] *= 0.1
    parts["b5"] = np.array([1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0])
    return pack(parts)
