"""Trains the learned initial-pose proposal (lsgcpd_proposal_*) and writes its
parameters.

The training pairs are registered by LSG-CPD itself: each pair (a scene of
2-3 primitives sampled twice, the source rotated uniformly on SO(3), noise
and outliers) is registered from its ground-truth pose by the batched
library call, and that solution is the pair's label.  The encoder's inputs
are each cloud in its own principal-axis frame, which does not change when a
cloud is rotated, so every pair is one training example (rotating it again
would give the same example).  The pairs are drawn in worker processes (host
only) and the arithmetic runs in the library's kernels; this script keeps
the loop.

  python -m paper_2103_15039_amd.train_proposal --out proposal_theta.npy

Prints one progress line every `--log` steps and a final summary (the
proposal's rotation error on held-out pairs).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def init_theta(rng):
    """He-uniform weights, zero biases; the last layer scaled by 0.1, its bias
    the identity rotation (first two columns e_x, e_y) and zero translation."""
    sizes = [(64, 3), (64,), (128, 64), (128,), (256, 128), (256,), (128, 512), (128,),
             (9, 128), (9,)]
    parts = []
    for i, s in enumerate(sizes):
        if len(s) == 2:
            w = rng.uniform(-1.0, 1.0, s) * math.sqrt(6.0 / s[1])
            parts.append(w * (0.1 if i == 8 else 1.0))
        elif i == 9:
            parts.append(np.array([1.0, 0, 0, 0, 1.0, 0, 0, 0, 0]))
        else:
            parts.append(np.zeros(s))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def angle_deg(A, B):
    """Rotation angle of A^T B (batched), by atan2."""
    D = np.einsum("nji,njk->nik", A, B)
    s = 0.5 * np.linalg.norm(np.stack([D[:, 2, 1] - D[:, 1, 2], D[:, 0, 2] - D[:, 2, 0],
                                       D[:, 1, 0] - D[:, 0, 1]], 1), axis=1)
    c = 0.5 * (np.trace(D, axis1=1, axis2=2) - 1.0)
    return np.degrees(np.arctan2(s, c))


def label_pairs(L, torch, pairs, iters, chunk=512):
    """LSG-CPD solutions of the pairs started from their ground truth."""
    R = np.empty((len(pairs), 3, 3))
    t = np.empty((len(pairs), 3))
    for i0 in range(0, len(pairs), chunk):
        part = pairs[i0:i0 + chunk]
        dev = [(torch.from_numpy(p.X).cuda(), torch.from_numpy(p.Y).cuda()) for p in part]
        res = L.register_batch(dev, k=10, max_iter=iters, init=[(p.R_gt, p.t_gt) for p in part])
        for j, r in enumerate(res):
            R[i0 + j], t[i0 + j] = r.R, r.t
    return R, t


def inputs(L, torch, pairs, P, chunk=1024):
    Xs, Ys, Ns = [], [], []
    for i0 in range(0, len(pairs), chunk):
        part = pairs[i0:i0 + chunk]
        Xn, Yn, nm = L.proposal_inputs([(torch.from_numpy(p.X).cuda(), torch.from_numpy(p.Y).cuda())
                                        for p in part], P)
        Xs.append(Xn)
        Ys.append(Yn)
        Ns.append(nm)
    return torch.cat(Xs).contiguous(), torch.cat(Ys).contiguous(), torch.cat(Ns).contiguous()


def _gen(args):
    """Proposal pairs of one chunk (worker process: host arrays only)."""
    import datagen
    n, trial, nmin, nmax = args
    return [(p.X, p.Y, p.R_gt, p.t_gt) for p in
            datagen.proposal_pairs(n, split="train", trial=trial, nmin=nmin, nmax=nmax)]


def make_pairs(n, seed, nmin, nmax, workers, chunk=1000):
    """n training pairs, chunk i drawn with trial seed * 100000 + i."""
    from types import SimpleNamespace
    jobs = [(min(chunk, n - i0), seed * 100000 + i0 // chunk, nmin, nmax)
            for i0 in range(0, n, chunk)]
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            parts = pool.map(_gen, jobs)
    else:
        parts = [_gen(j) for j in jobs]
    return [SimpleNamespace(X=X, Y=Y, R_gt=R, t_gt=t) for part in parts for X, Y, R, t in part]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=50000, help="training pairs (one LSG-CPD solve each)")
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--points", type=int, default=512)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--label-iters", type=int, default=30)
    ap.add_argument("--nmin", type=int, default=1000)
    ap.add_argument("--nmax", type=int, default=4000)
    ap.add_argument("--holdout", type=int, default=512)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--log", type=int, default=1000)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)

    t0 = time.time()
    pairs = make_pairs(a.pairs, a.seed, a.nmin, a.nmax, a.workers)
    hold = make_pairs(a.holdout, a.seed + 1, a.nmin, a.nmax, 1)
    print(json.dumps({"stage": "pairs", "pairs": len(pairs), "s": round(time.time() - t0, 1)}),
          flush=True)
    import torch
    import paper_2103_15039_amd as L

    Rl, tl = label_pairs(L, torch, pairs, a.label_iters)
    drift = angle_deg(np.stack([p.R_gt for p in pairs]), Rl)
    print(json.dumps({"stage": "labels", "s": round(time.time() - t0, 1),
                      "label_vs_truth_deg_median": float(np.median(drift)),
                      "label_vs_truth_deg_max": float(drift.max())}), flush=True)
    Xn, Yn, norm = inputs(L, torch, pairs, a.points)
    hX, hY, hN = inputs(L, torch, hold, a.points)
    hR = np.stack([p.R_gt for p in hold])
    labels = np.concatenate([Rl.reshape(-1, 9), tl], axis=1)
    del pairs

    rng = np.random.default_rng([2103, 15039, a.seed])
    theta = torch.from_numpy(init_theta(rng)).cuda()
    m, v = torch.zeros_like(theta), torch.zeros_like(theta)
    n = len(labels)
    hist = []
    t1 = time.time()
    for step in range(1, a.steps + 1):
        idx = rng.integers(0, n, a.batch).astype(np.int32)
        lr = a.lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / a.steps)))
        loss, _, _ = L.proposal_train_step(theta, m, v, step, lr, Xn, Yn, norm, labels[idx],
                                           index=idx)
        hist.append(float(loss.mean()))
        if step % a.log == 0 or step == a.steps:
            pose = L.proposal_forward(theta, hX, hY, hN).cpu().numpy()
            err = angle_deg(hR, pose[:, :9].reshape(-1, 3, 3))
            print(json.dumps({"step": step, "of": a.steps, "lr": lr,
                              "loss": float(np.mean(hist[-a.log:])),
                              "holdout_rot_err_deg_median": float(np.median(err)),
                              "holdout_within_30deg": float(np.mean(err < 30)),
                              "holdout_within_60deg": float(np.mean(err < 60)),
                              "s": round(time.time() - t1, 1)}), flush=True)
    np.save(a.out, theta.cpu().numpy())
    print(json.dumps({"stage": "done", "out": a.out, "steps": a.steps,
                      "examples_seen": a.steps * a.batch, "s": round(time.time() - t0, 1)}),
          flush=True)


if __name__ == "__main__":
    main()
