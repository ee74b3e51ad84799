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
    s = root-mean-square distance of the sampled y from mu_Y (s = 1 when the
    target's samples are all one point, e.g. P = 1);
  * each cloud's principal-axis frame F = [e0 e1 e2]: the eigenvectors of
    the covariance of its centred samples (1/P), eigenvalues in decreasing
    order; e0 and e1 signed so that the third moment of the samples along
    them is >= 0 (if it is exactly 0, so that their largest component is
    positive), e2 = e0 x e1; F = I if the covariance is zero;
  * inputs F_X^T (x' - mu_X) / s and F_Y^T (y - mu_Y) / s: both clouds in
    their own frames, so the inputs do not change when either cloud is
    rotated, and what is left to predict is the rotation between the frames.
A pose (R, t) mapping x' onto y reads, in these units, R_c = F_Y^T R F_X and
t^ = F_Y^T (R mu_X + t - mu_Y) / s; a prediction (R_c, t^) maps back to
R = F_Y R_c F_X^T, t = mu_Y + s F_Y t^ - R mu_X.
Loss of a pair: |a1 - R_c e_x|^2 + |a2 - R_c e_y|^2 + |t^ - t^_label|^2, with
a1, a2 the two 3-vectors of the output and R_c the label's rotation in the
frames -- least squares on the 6-D representation itself (the rotation it
gives by Gram-Schmidt is the prediction).  A loss on the rotation would have
no gradient where the prediction is a half turn from the label, which is
where the frames' sign choices leave many labels; of a batch: the mean.
Optimiser: Adam (Kingma and Ba, ICLR 2015) with bias correction,
beta1 = 0.9, beta2 = 0.999, eps = 1e-8.

Max-pool ties go to the lower point index.  Where a channel's largest
activation is 0 (every point inactive), its gradient is 0.

Parity status: pinned by tests/test_oracle_proposal.py -- Gram-Schmidt against
its closed-form properties, the forward pass against an independent float64
implementation in torch, every gradient against central finite differences
(the loss is also pinned at the label, 0, and its minimiser),
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


def principal_frame(c):
    """Principal-axis frame of centred points c (P x 3), signs as stated in
    the module docstring."""
    C = c.T @ c / len(c)
    if not np.any(C):
        return np.eye(3)
    w, V = np.linalg.eigh(C)
    V = V[:, ::-1].copy()
    for a in range(2):
        m3 = np.sum((c @ V[:, a]) ** 3)
        if m3 < 0.0 or (m3 == 0.0 and V[np.argmax(np.abs(V[:, a])), a] < 0.0):
            V[:, a] = -V[:, a]
    V[:, 2] = np.cross(V[:, 0], V[:, 1])
    return V


def normalise(X, Y, P, Q=None):
    """Encoder inputs of one pair and the normalisation (mu_X, mu_Y, s, F_X,
    F_Y)."""
    xs = np.asarray(X, np.float64)[sample_indices(len(X), P)]
    ys = np.asarray(Y, np.float64)[sample_indices(len(Y), P)]
    if Q is not None:
        xs = xs @ np.asarray(Q, np.float64).T
    mx, my = xs.mean(axis=0), ys.mean(axis=0)
    s = np.sqrt(np.mean(np.sum((ys - my) ** 2, axis=1)))
    if not s > 0.0:
        s = 1.0  # the target's samples are one point: no scale to take
    FX, FY = principal_frame(xs - mx), principal_frame(ys - my)
    return (xs - mx) @ FX / s, (ys - my) @ FY / s, (mx, my, s, FX, FY)


def label_normalised(R, t, norm):
    """(R_c, t^) of a pose mapping x' onto y, in the units of norm."""
    mx, my, s, FX, FY = norm
    R = np.asarray(R, np.float64)
    return FY.T @ R @ FX, FY.T @ (R @ mx + np.asarray(t) - my) / s


def pose_from_prediction(R_c, t_hat, norm):
    """World pose of a prediction in the units of norm."""
    mx, my, s, FX, FY = norm
    R = FY @ np.asarray(R_c, np.float64) @ FX.T
    return R, my + s * (FY @ np.asarray(t_hat)) - R @ mx


def gram_schmidt(a1, a2):
    """Rotation whose columns are a1 normalised, the part of a2 orthogonal to
    it normalised, and their cross product."""
    b1 = a1 / np.linalg.norm(a1)
    u2 = a2 - (b1 @ a2) * b1
    b2 = u2 / np.linalg.norm(u2)
    b3 = np.cross(b1, b2)
    return np.stack([b1, b2, b3], axis=1)


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


def pair_target(R_l, t_l):
    """The 9 outputs a pair's label asks for: R_l's first two columns, t_l."""
    R_l = np.asarray(R_l, np.float64)
    return np.concatenate([R_l[:, 0], R_l[:, 1], np.asarray(t_l, np.float64)])


def pair_loss(pp, R_l, t_l):
    return float(np.sum((pp.o - pair_target(R_l, t_l)) ** 2))


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
        go = 2.0 * (pp.o - pair_target(R_l[i], t_l[i])) / B
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
