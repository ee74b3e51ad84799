"""Plain, slow FP64 reference for LSG-CPD (Liu, Wu, Chirikjian, "LSG-CPD: Coherent
Point Drift with Local Surface Geometry for Point Cloud Registration", ICCV 2021).

TEST INFRASTRUCTURE ONLY.  This module is the oracle that the GPU library is
checked against.  Only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark may import it; the library itself never does, and nothing here
is shared with the GPU code (no kernels, headers, constants or helpers).

Every function evaluates the paper's definitions directly in float64, in the
paper's notation:

  X (N x 3)  source points x_n        Y (M x 3)  target points y_m
  normals    unit normals n_m          alpha      penalty alpha_m  (Eq. 3)
  w          outlier weights w_n       pi         priors pi(m)
  g = (R, t) rigid transform, g(x) = R x + t (maps the source onto the target)

Inputs that arrive as float32 are promoted exactly to float64 before any
arithmetic.  Where the paper is silent or ambiguous the reading taken is stated
at the function that takes it.

Parity status: every function here is pinned by the CPU test-suite
(tests/test_oracle_*.py) against closed forms, brute force, special cases that
reduce to textbook routines (rigid CPD, weighted Procrustes), finite
differences, or invariants.  The 86 lifted statistics are pinned by the
quadratic they encode: D(G) rebuilt from them equals the dense double sum of
P_mn d_mn(G) at arbitrary 3 x 4 matrices G, and its derivatives along SE(3)
are Eq. (11)-(12) as printed.  Not pinned: the surface normal at a repeated
smallest eigenvalue, which is not unique ("parity unpinned": only n n^T at a
clear eigengap is compared).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

_CHUNK = 1 << 22  # pairs per chunk of the dense (m, n) loops (memory bound only)


def _f64(a):
    return np.asarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
# Target geometry: neighbourhoods, surface normal, surface variation, penalty
# ----------------------------------------------------------------------------

def knn_indices(Y, k, queries=None):
    """k nearest targets of each query target, the query itself included.

    Sec. 3.1 (surface variation of a local neighbourhood of y_m).  The paper
    does not say how the neighbourhood is formed; reading: the k nearest
    points of Y by Euclidean distance, the point itself included, ties broken
    by the lower index.  The distance decides an integer (which points are
    neighbours), so it is taken in float32, the precision of the input cloud,
    as ((dx*dx + dy*dy) + dz*dz) with every operation rounded to float32 and
    no fused multiply-add.  Full stable argsort = brute force.

    Returns int64 (Q, k), rows ordered by (distance, index).
    """
    Y32 = np.asarray(Y, dtype=np.float32)
    M = Y32.shape[0]
    if not (1 <= k <= M):
        raise ValueError("need 1 <= k <= M")
    q = np.arange(M) if queries is None else np.asarray(queries, dtype=np.int64)
    out = np.empty((q.size, k), dtype=np.int64)
    rows = max(1, _CHUNK // max(M, 1))
    for s in range(0, q.size, rows):
        qi = q[s:s + rows]
        d = np.zeros((qi.size, M), dtype=np.float32)
        dd = []
        for c in range(3):
            dc = (Y32[qi, c][:, None] - Y32[None, :, c]).astype(np.float32)
            dd.append((dc * dc).astype(np.float32))
        d = ((dd[0] + dd[1]).astype(np.float32) + dd[2]).astype(np.float32)
        order = np.argsort(d, axis=1, kind="stable")
        out[s:s + rows] = order[:, :k]
    return out


def local_geometry(Y, nbr):
    """Surface normal n_m and surface variation kappa_m of each neighbourhood.

    Sec. 3.1: kappa is the smallest eigenvalue of the neighbourhood covariance
    divided by its trace (kappa in [0, 1/3]); the normal is the eigenvector of
    that smallest eigenvalue (Pauly et al.; Hoppe et al.).  Covariance is taken
    about the neighbourhood centroid with weight 1/k (reading).  Degenerate
    neighbourhood (trace 0, all neighbours coincide): kappa = 1/3, n = e_z
    (reading).  Eigen-decomposition: numpy.linalg.eigh.
    """
    Y = _f64(Y)
    P = Y[nbr]                                     # (M, k, 3)
    c = P.mean(axis=1, keepdims=True)
    D = P - c
    C = np.einsum("mki,mkj->mij", D, D) / nbr.shape[1]
    lam, vec = np.linalg.eigh(C)                   # ascending eigenvalues
    tr = np.trace(C, axis1=1, axis2=2)
    n = vec[:, :, 0].copy()
    kappa = np.empty(nbr.shape[0])
    deg = tr <= 0.0
    kappa[~deg] = lam[~deg, 0] / tr[~deg]
    kappa[deg] = 1.0 / 3.0
    n[deg] = (0.0, 0.0, 1.0)
    kappa = np.clip(kappa, 0.0, 1.0 / 3.0)
    return n, kappa, lam, tr


def penalty_alpha(kappa, alpha_max, lam):
    """Adaptive point-to-plane penalty alpha_m, Eq. (3), the modified logistic
    of 1/kappa_m.  kappa = 0 takes the stated limit alpha_max; values are
    clamped at 0 so that rounding at kappa = 1/3 cannot make alpha negative
    (reading)."""
    kappa = _f64(kappa)
    out = np.empty_like(kappa)
    zero = kappa <= 0.0
    out[zero] = alpha_max
    kz = kappa[~zero]
    with np.errstate(over="ignore"):
        u = np.exp(lam * (3.0 - 1.0 / kz))
        a = (1.0 - u) / (1.0 + u) * alpha_max
    a[np.isinf(u)] = -alpha_max   # exp overflow cannot occur for kappa <= 1/3
    out[~zero] = a
    return np.maximum(out, 0.0)


def normals(Y, k, alpha_max, lam):
    """Normals, surface variation and penalty for every target point
    (Sec. 3.1 and Eq. 3)."""
    nbr = knn_indices(Y, k)
    n, kappa, _, _ = local_geometry(Y, nbr)
    return n, kappa, penalty_alpha(kappa, alpha_max, lam)


# ----------------------------------------------------------------------------
# Model set-up: working volume, initial variance
# ----------------------------------------------------------------------------

def working_volume(Y):
    """Volume V of the working space that holds the target (Sec. 3.1, uniform
    outlier density p_o = 1/V).  The paper leaves the solid unspecified;
    reading: the target's axis-aligned bounding box, each edge floored at
    1e-3 of the box diagonal (a unit box if the target is a single point)."""
    Y = _f64(Y)
    ext = Y.max(axis=0) - Y.min(axis=0)
    diag = math.sqrt(float(ext @ ext))
    if diag == 0.0:
        return 1.0
    ext = np.maximum(ext, 1e-3 * diag)
    return float(ext[0] * ext[1] * ext[2])


def bbox_diag(Y):
    Y = _f64(Y)
    ext = Y.max(axis=0) - Y.min(axis=0)
    return math.sqrt(float(ext @ ext))


def sigma2_init(X, Y, R, t):
    """Initial covariance multiplier (Sec. 3.1: set automatically as in CPD).
    Reading: CPD's rule with D = 3, the mean squared distance over all
    (m, n) pairs divided by 3:  sum_mn ||g(x_n) - y_m||^2 / (3 M N)."""
    Xg = _f64(X) @ _f64(R).T + _f64(t)
    Y = _f64(Y)
    tot = 0.0
    rows = max(1, _CHUNK // max(Xg.shape[0], 1))
    for s in range(0, Y.shape[0], rows):
        d = Y[s:s + rows, None, :] - Xg[None, :, :]
        tot += float(np.sum(d * d))
    return tot / (3.0 * Y.shape[0] * Xg.shape[0])


# ----------------------------------------------------------------------------
# E step
# ----------------------------------------------------------------------------

@dataclass
class EStep:
    """Dense E-step result.  P[m, n] as in Eq. (5)/(9)."""
    P: np.ndarray            # (M, N) posterior of x_n belonging to component m
    Ksum: np.ndarray         # (N,) sum_m K_mn
    gamma: float             # (2 pi sigma^2)^{3/2} / V
    nll: float               # Eq. (4) at the pose used
    sigma2: float
    V: float


def _prior_arrays(M, N, pi, w, w0):
    pi = np.full(M, 1.0 / M) if pi is None else _f64(pi)
    w = np.full(N, float(w0)) if w is None else _f64(w)
    return pi, w


def mahalanobis_sq(Xg, Y, normals, alpha):
    """d_mn = (g(x_n) - y_m)^T (alpha_m n_m n_m^T + I) (g(x_n) - y_m), i.e.
    sigma^2 times the quadratic form of Eq. (2).  Dense (M, N)."""
    Y = _f64(Y)
    nrm = _f64(normals)
    a = _f64(alpha)
    r = Xg[None, :, :] - Y[:, None, :]                 # (M, N, 3)
    q = np.einsum("mnk,mnk->mn", r, r)
    p = np.einsum("mnk,mk->mn", r, nrm)
    return q + a[:, None] * p * p


def estep(X, Y, normals, alpha, R, t, sigma2, w0=None, V=None, pi=None, w=None,
          exact_normalizer=False):
    """Posterior of every (component m, source point n) pair.

    Eq. (5) with the component density of Eq. (2), written in the form of
    Eq. (9):  P_mn = K_mn / (sum_m K_mn + gamma),
    K_mn = (1 - w_n)/w_n * pi(m) * exp(-d_mn / (2 sigma^2)),
    gamma = (2 pi sigma^2)^{3/2} / V.
    The printed Eq. (9) takes the component normaliser as (2 pi sigma^2)^{-3/2};
    a true Gaussian with the covariance of Eq. (2) has the extra factor
    sqrt(1 + alpha_m).  Default: as printed; exact_normalizer=True multiplies
    K_mn by sqrt(1 + alpha_m) (reading).  p_o = 1/V is used for every point
    (reading of the working-space definition, as in Eq. 9).  Requires
    0 < w_n < 1.  Also returns the negative log-likelihood of Eq. (4):
    -sum_n log( w_n / V + (1 - w_n) sum_m pi(m) p(g(x_n)|m) ).
    """
    X = _f64(X)
    Y = _f64(Y)
    M, N = Y.shape[0], X.shape[0]
    pi, w = _prior_arrays(M, N, pi, w, w0)
    if np.any(w <= 0) or np.any(w >= 1):
        raise ValueError("outlier weights must lie in (0, 1)")
    if V is None:
        V = working_volume(Y)
    Xg = X @ _f64(R).T + _f64(t)
    d = mahalanobis_sq(Xg, Y, normals, alpha)
    C = ((1.0 - w) / w)[None, :] * pi[:, None]
    if exact_normalizer:
        C = C * np.sqrt(1.0 + _f64(alpha))[:, None]
    K = C * np.exp(-d / (2.0 * sigma2))
    gamma = (2.0 * math.pi * sigma2) ** 1.5 / V
    Ksum = K.sum(axis=0)
    P = K / (Ksum + gamma)[None, :]
    # Eq. (4): p(g(x_n)) = w_n (2 pi s2)^{-3/2} (Ksum_n + gamma)
    nll = -float(np.sum(np.log(w) + np.log(Ksum + gamma)
                        - 1.5 * math.log(2.0 * math.pi * sigma2)))
    return EStep(P=P, Ksum=Ksum, gamma=gamma, nll=nll, sigma2=sigma2, V=V)


# ----------------------------------------------------------------------------
# Per-source aggregates of the posterior (sums over m for each source n)
# ----------------------------------------------------------------------------

@dataclass
class Columns:
    """Sums over the components m of P-weighted quantities, one per source n.

    With M_m = I + alpha_m n_m n_m^T (sigma^2 Sigma_m^{-1} of Eq. 2):
      p[n]   = sum_m P_mn
      A[n]   = sum_m P_mn M_m                (3 x 3)
      B[n]   = sum_m P_mn M_m y_m            (3)
      C[n]   = sum_m P_mn y_m^T M_m y_m
      b[n]   = sum_m P_mn M_m (g(x_n) - y_m) (3)   at the E-step pose
      c[n]   = sum_m P_mn d_mn                     at the E-step pose
    """
    p: np.ndarray
    A: np.ndarray
    B: np.ndarray
    C: np.ndarray
    b: np.ndarray
    c: np.ndarray


def columns(P, X, Y, normals, alpha, R, t):
    """Per-source aggregates of a dense posterior (see Columns).  These are
    the sums over m inside Eq. (11)-(12) and inside Q of Eq. (6), taken for
    each n (linearity of the double sums)."""
    X = _f64(X)
    Y = _f64(Y)
    nrm = _f64(normals)
    a = _f64(alpha)
    Mm = np.eye(3)[None] + a[:, None, None] * nrm[:, :, None] * nrm[:, None, :]
    p = P.sum(axis=0)
    A = np.einsum("mn,mij->nij", P, Mm)
    My = np.einsum("mij,mj->mi", Mm, Y)
    B = P.T @ My
    C = P.T @ np.einsum("mi,mi->m", Y, My)
    Xg = X @ _f64(R).T + _f64(t)
    b = np.einsum("nij,nj->ni", A, Xg) - B
    d = mahalanobis_sq(Xg, Y, normals, alpha)
    c = np.einsum("mn,mn->n", P, d)
    return Columns(p=p, A=A, B=B, C=C, b=b, c=c)


# ----------------------------------------------------------------------------
# M step on SE(3)
# ----------------------------------------------------------------------------

def se3_basis():
    """Basis E_1..E_6 of se(3) as 4x4 matrices: E_1..E_3 rotate about the x, y,
    z axes, E_4..E_6 translate along them (Sec. 3.5; the ordering is a
    reading, it does not change the step)."""
    E = np.zeros((6, 4, 4))
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1.0
        E[i, :3, :3] = hat3(e)
        E[3 + i, i, 3] = 1.0
    return E


def hat3(w):
    w = _f64(w)
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_hat(xi):
    """The wedge map of Sec. 3.5: 6-vector -> element of se(3)."""
    return np.einsum("i,ijk->jk", _f64(xi), se3_basis())


def se3_exp(xi):
    """Matrix exponential of se3_hat(xi) in closed form (rotation by the
    Rodrigues formula, translation by the left Jacobian of SO(3)); series
    coefficients for small angles."""
    xi = _f64(xi)
    w, v = xi[:3], xi[3:]
    th = math.sqrt(float(w @ w))
    W = hat3(w)
    W2 = W @ W
    if th < 1e-6:
        A = 1.0 - th * th / 6.0
        B = 0.5 - th * th / 24.0
        Cc = 1.0 / 6.0 - th * th / 120.0
    else:
        A = math.sin(th) / th
        B = (1.0 - math.cos(th)) / (th * th)
        Cc = (th - math.sin(th)) / (th ** 3)
    Rm = np.eye(3) + A * W + B * W2
    Vm = np.eye(3) + B * W + Cc * W2
    T = np.eye(4)
    T[:3, :3] = Rm
    T[:3, 3] = Vm @ v
    return T


def homog(R, t):
    T = np.eye(4)
    T[:3, :3] = _f64(R)
    T[:3, 3] = _f64(t)
    return T


def grad_hess_literal(P, X, Y, normals, alpha, R, t, sigma2):
    """Eq. (11) and Eq. (12) exactly as printed: double sums over (m, n) with
    homogeneous g~, x~_n, y~_m and Sigma~^{-1}_m = Sigma_m^{-1} (+) 0.
    O(M N) dense; meant for small clouds."""
    X = _f64(X)
    Y = _f64(Y)
    nrm = _f64(normals)
    a = _f64(alpha)
    M, N = Y.shape[0], X.shape[0]
    E = se3_basis()
    g = homog(R, t)
    xt = np.hstack([X, np.ones((N, 1))])
    yt = np.hstack([Y, np.ones((M, 1))])
    S = np.zeros((M, 4, 4))
    S[:, :3, :3] = (np.eye(3)[None] + a[:, None, None] * nrm[:, :, None] * nrm[:, None, :]) / sigma2
    grad = np.zeros(6)
    H = np.zeros((6, 6))
    gEx = np.einsum("ab,ibc,nc->ina", g, E, xt)            # g E_i x~_n  (6, N, 4)
    gEEx = np.einsum("ab,jbc,icd,nd->jina", g, E, E, xt)   # g E_j E_i x~_n (6,6,N,4)
    for m in range(M):
        r = (xt @ g.T) - yt[m]                             # (N, 4)
        Sr = r @ S[m]                                      # (N, 4) = r^T Sigma~
        Pm = P[m]
        for i in range(6):
            grad[i] += 2.0 * np.sum(Pm * np.einsum("na,na->n", Sr, gEx[i]))
        SgEx = np.einsum("ab,inb->ina", S[m], gEx)        # Sigma~ g E_i x~
        for i in range(6):
            for j in range(6):
                t1 = np.einsum("na,na->n", gEx[j], SgEx[i])
                t2 = np.einsum("na,na->n", Sr, gEEx[j, i])
                H[i, j] += 2.0 * np.sum(Pm * (t1 + t2))
    return grad, H


def grad_hess(cols, X, R, t, sigma2):
    """Eq. (11) and Eq. (12) with the sum over m taken first for each n, using
    the per-source aggregates A[n], B[n] (linearity):
      sum_m P_mn Sigma_m^{-1}(g x_n - y_m) = (A[n] g(x_n) - B[n]) / sigma^2,
      sum_m P_mn Sigma_m^{-1}              =  A[n] / sigma^2."""
    X = _f64(X)
    N = X.shape[0]
    E = se3_basis()
    g = homog(R, t)
    xt = np.hstack([X, np.ones((N, 1))])
    xg = xt @ g.T                                          # g~ x~_n, (N, 4)
    u = (np.einsum("nij,nj->ni", cols.A, xg[:, :3]) - cols.B) / sigma2   # (N, 3)
    gEx = np.einsum("ab,ibc,nc->ina", g, E, xt)[:, :, :3]  # (6, N, 3)
    gEEx = np.einsum("ab,jbc,icd,nd->jina", g, E, E, xt)[:, :, :, :3]
    grad = 2.0 * np.einsum("ni,kni->k", u, gEx)
    AgEx = np.einsum("nab,knb->kna", cols.A, gEx) / sigma2
    H = 2.0 * (np.einsum("jna,ina->ij", gEx, AgEx)
               + np.einsum("na,jina->ij", u, gEEx))
    return grad, H


def pd_of(cols, X, R, t):
    """sum_mn P_mn d_mn(g) for the posterior behind `cols`, from the
    per-source aggregates:  sum_n [x'^T A x' - 2 x'^T B + C],  x' = g(x_n)."""
    Xg = _f64(X) @ _f64(R).T + _f64(t)
    return float(np.sum(np.einsum("ni,nij,nj->n", Xg, cols.A, Xg)
                        - 2.0 * np.einsum("ni,ni->n", Xg, cols.B) + cols.C))


def nll_terms(es, w=None, w0=None):
    """The three E-step by-products that complete the 86 statistics: the sum
    over sources of log(sum_m K_mn + gamma), the outlier mass
    sum_n gamma / (sum_m K_mn + gamma) (the outlier posterior of each source,
    Eq. 5/9), and sum_n log w_n.  With them the negative log-likelihood of
    Eq. (4) is  -(t[2] + t[0] - (3/2) N log(2 pi sigma^2))."""
    w = np.full(es.Ksum.shape[0], float(w0)) if w is None else _f64(w)
    den = es.Ksum + es.gamma
    return [float(np.sum(np.log(den))), float(np.sum(es.gamma / den)),
            float(np.sum(np.log(w)))]


def lifted_stats(cols, X, nll_terms=None):
    """The 86 sufficient statistics the GPU library reports for one E step,
    written from their definitions (x~_n = (x_n, 1), p, W = A - p I, B, C the
    per-source aggregates of Columns):
      S0 = sum_n p_n x~ x~^T, S1[ab] = sum_n W_n[a,b] x~ x~^T (ab = 00 01 02 11
      12 22), S2 = sum_n B_n x~^T, S3 = sum_n C_n, then the three NLL terms.
    Upper-triangle order of a 4x4: 00 01 02 03 11 12 13 22 23 33."""
    X = _f64(X)
    xt = np.hstack([X, np.ones((X.shape[0], 1))])
    iu = [(i, j) for i in range(4) for j in range(i, 4)]
    xx = np.stack([xt[:, i] * xt[:, j] for (i, j) in iu], axis=1)     # (N, 10)
    W = cols.A - cols.p[:, None, None] * np.eye(3)[None]
    out = np.zeros(86)
    out[0:10] = cols.p @ xx
    for k, (a, b) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        out[10 + 10 * k:20 + 10 * k] = W[:, a, b] @ xx
    out[70:82] = (cols.B.T @ xt).reshape(12)
    out[82] = float(np.sum(cols.C))
    if nll_terms is not None:
        out[83:86] = nll_terms
    return out


@dataclass
class MStep:
    R: np.ndarray
    t: np.ndarray
    sigma2: float
    newton_iters: int
    gn_fallbacks: int


def mstep(cols, X, R, t, sigma2, newton_max=20, sigma2_floor=0.0):
    """M step of Sec. 3.5: minimise Q of Eq. (6) over g on SE(3) by Newton's
    method with the symmetrised Hessian (H + H^T)/2 (Eq. 12-13), then set
    sigma^2 where dQ/dsigma^2 = 0 at the new g.

    Readings: Eq. (13) is read as g <- g exp(xi^) with
    xi = -((H + H^T)/2)^{-1} grad (descent direction); Newton is run to
    convergence inside one M step (|xi|_inf < 1e-12 or newton_max steps); if
    (H + H^T)/2 is not positive definite its first (Gauss-Newton) term is used;
    the step is halved until Q does not increase by more than a rounding
    allowance of 1e-12 |Q| (at most 30 halvings).
    sigma^2 = sum_mn P_mn d_mn(g_new) / (3 sum_mn P_mn), not below sigma2_floor.
    """
    Np = float(np.sum(cols.p))
    R = _f64(R).copy()
    t = _f64(t).copy()
    if Np <= 0.0:
        return MStep(R, t, sigma2, 0, 0)
    g = homog(R, t)
    cur = pd_of(cols, X, g[:3, :3], g[:3, 3])
    it = 0
    gnf = 0
    E = se3_basis()
    N = _f64(X).shape[0]
    xt = np.hstack([_f64(X), np.ones((N, 1))])
    while it < newton_max:
        it += 1
        grad, H = grad_hess(cols, X, g[:3, :3], g[:3, 3], sigma2)
        Hs = 0.5 * (H + H.T)
        try:
            L = np.linalg.cholesky(Hs)
            xi = -np.linalg.solve(Hs, grad)
        except np.linalg.LinAlgError:
            gnf += 1
            gEx = np.einsum("ab,ibc,nc->ina", g, E, xt)[:, :, :3]
            AgEx = np.einsum("nab,knb->kna", cols.A, gEx) / sigma2
            Hg = 2.0 * np.einsum("jna,ina->ij", gEx, AgEx)
            Hg = 0.5 * (Hg + Hg.T)
            xi = -np.linalg.lstsq(Hg, grad, rcond=None)[0]
        step = 1.0
        accepted = False
        for _ in range(31):
            gn = g @ se3_exp(step * xi)
            val = pd_of(cols, X, gn[:3, :3], gn[:3, 3])
            if val <= cur + 1e-12 * abs(cur):
                accepted = True
                break
            step *= 0.5
        if not accepted:
            break
        g = gn
        cur = val
        if np.max(np.abs(step * xi)) < 1e-12:
            break
    s2 = max(cur / (3.0 * Np), sigma2_floor)
    return MStep(g[:3, :3].copy(), g[:3, 3].copy(), s2, it, gnf)


# ----------------------------------------------------------------------------
# Outlier weight from the outlier ratio (Sec. 3.2), confidence filtering (Sec. 3.3)
# ----------------------------------------------------------------------------

def component_peak(alpha, sigma2, exact_normalizer=False):
    """c_m: the largest value of the component density p(x|m) of Eq. (2), i.e.
    its value at x = y_m.  With the normaliser the E step uses (Eq. 9) this is
    (2 pi sigma^2)^{-3/2} for every m; with exact_normalizer it is the true
    Gaussian's sqrt(det Sigma_m^{-1}) / (2 pi)^{3/2} = sqrt(1 + alpha_m) (2 pi
    sigma^2)^{-3/2} (reading: c_m is taken for the same density the E step
    evaluates, so that p(x|m) <= c_m holds for it)."""
    a = _f64(alpha)
    c = np.full(a.shape, (2.0 * math.pi * sigma2) ** -1.5)
    if exact_normalizer:
        c = c * np.sqrt(1.0 + a)
    return c


def outlier_weight_max(eta, V, pi, alpha, sigma2, exact_normalizer=False):
    """Sec. 3.2: the largest uniform outlier weight consistent with an expected
    outlier count of eta N, w_max = eta V S / ((1 - eta) + eta V S) with
    S = sum_m pi(m) c_m.  c_m depends on sigma^2, so w_max does too; register
    evaluates it once, at the initial sigma^2, and keeps w0 fixed (reading:
    re-evaluating it as sigma^2 shrinks would drive w0 towards 1, the regime
    Sec. 3.2 warns against).  pi None => uniform 1/M.  Requires 0 <= eta < 1."""
    if not (0.0 <= eta < 1.0):
        raise ValueError("eta must lie in [0, 1)")
    a = _f64(alpha)
    pi = np.full(a.shape, 1.0 / a.shape[0]) if pi is None else _f64(pi)
    S = float(np.sum(pi * component_peak(a, sigma2, exact_normalizer)))
    return eta * V * S / ((1.0 - eta) + eta * V * S)


def depth_confidence(P, coef, e_min):
    """Sec. 3.3: measurement confidence phi(x) = e_min / e(x) of a point seen by
    a depth sensor, with the error model e(x) = c0 + c1 z + c2 z^2 of its depth
    z = x_3 in the sensor frame.  The paper leaves the model to the sensor;
    this quadratic-in-depth form is the reading.  Points whose modelled error
    is below e_min (outside the range e_min was taken over) get phi = 1."""
    z = _f64(P)[:, 2]
    c0, c1, c2 = (float(c) for c in coef)
    e = c0 + c1 * z + c2 * z * z
    out = np.ones_like(e)
    far = e > float(e_min)
    out[far] = float(e_min) / e[far]
    return out


def confidence_priors(phi_y, phi_x, w0):
    """Sec. 3.3 (confidence filtering): component priors
    pi(m) = phi(y_m) / sum_m phi(y_m) and outlier weights
    w_n = 1 - (1 - w0) phi(x_n).  Either side may be None (uniform)."""
    pi = None if phi_y is None else _f64(phi_y) / float(np.sum(_f64(phi_y)))
    w = None if phi_x is None else 1.0 - (1.0 - float(w0)) * _f64(phi_x)
    return pi, w


def truncate(P, phi, threshold):
    """Sec. 3.3: the points whose confidence is at least `threshold`, in their
    original order, with their confidences."""
    keep = _f64(phi) >= float(threshold)
    return np.asarray(P)[keep], np.asarray(phi)[keep]


# ----------------------------------------------------------------------------
# EM driver
# ----------------------------------------------------------------------------

@dataclass
class Registration:
    R: np.ndarray
    t: np.ndarray
    sigma2: float
    iters: int
    nll: list = field(default_factory=list)       # Eq. (4) at each E step
    sigma2_trace: list = field(default_factory=list)
    R_trace: list = field(default_factory=list)
    t_trace: list = field(default_factory=list)
    gn_fallbacks: int = 0
    normals: np.ndarray | None = None
    alpha: np.ndarray | None = None
    V: float = 0.0
    N: int = 0                                    # points used (after truncation)
    M: int = 0
    w0: float = 0.0                               # uniform outlier weight used


def register(X, Y, k=10, alpha_max=30.0, lam=0.2, w0=0.1, max_iter=50, tol=0.0,
             R0=None, t0=None, sigma2_0=None, V=None, newton_max=20,
             exact_normalizer=False, target_normals=None, target_alpha=None,
             estep_columns=None, eta=None, phi_x=None, phi_y=None, cf_threshold=0.0):
    """LSG-CPD rigid registration by EM (Sec. 3): target normals and penalty
    (Sec. 3.1, Eq. 3), working volume and initial sigma^2, then alternate the
    E step (Eq. 5/9) and the M step (Sec. 3.5).

    Outlier weights and priors: w_n = w0 and pi(m) = 1/M, unless
      eta     -- w0 = w_max (Sec. 3.2) at the initial sigma^2;
      phi_x, phi_y -- confidences of the source and target points: confidence
                 filtering (Sec. 3.3), pi(m) proportional to phi(y_m) and
                 w_n = 1 - (1 - w0) phi(x_n);
      cf_threshold -- points whose confidence is below it are dropped first
                 (Sec. 3.3); normals, V and sigma^2_0 come from what is kept.
    Readings: a fixed number of iterations unless tol > 0, in which case EM stops once
    |L_i - L_{i-1}| <= tol |L_i| for the negative log-likelihood L of Eq. (4);
    sigma^2 is floored at 1e-12 times the squared target box diagonal.

    `estep_columns(R, t, sigma2)` may replace the dense E step by any routine
    that returns (Columns, nll) for the same definitions (used for clouds too
    large for a dense M x N matrix).
    """
    if cf_threshold > 0.0:
        if phi_x is not None:
            X, phi_x = truncate(X, phi_x, cf_threshold)
        if phi_y is not None:
            Y, phi_y = truncate(Y, phi_y, cf_threshold)
    if estep_columns is not None and (eta is not None or phi_x is not None
                                      or phi_y is not None):
        raise ValueError("estep_columns takes uniform priors and a fixed w0 only")
    X = _f64(X)
    Y = _f64(Y)
    if target_normals is None:
        nrm, _, alpha = normals(Y, k, alpha_max, lam)
    else:
        nrm, alpha = _f64(target_normals), _f64(target_alpha)
    R = np.eye(3) if R0 is None else _f64(R0).copy()
    t = np.zeros(3) if t0 is None else _f64(t0).copy()
    if V is None:
        V = working_volume(Y)
    s2 = sigma2_init(X, Y, R, t) if sigma2_0 is None else float(sigma2_0)
    floor = 1e-12 * bbox_diag(Y) ** 2
    out = Registration(R=R, t=t, sigma2=s2, iters=0, normals=nrm, alpha=alpha, V=V,
                       N=X.shape[0], M=Y.shape[0])
    pi, _ = confidence_priors(phi_y, None, w0)
    if eta is not None:
        w0 = outlier_weight_max(eta, V, pi, alpha, s2, exact_normalizer)
    _, w = confidence_priors(None, phi_x, w0)
    out.w0 = w0
    prev = None
    for it in range(max_iter):
        if estep_columns is None:
            es = estep(X, Y, nrm, alpha, R, t, s2, w0=w0, V=V, pi=pi, w=w,
                       exact_normalizer=exact_normalizer)
            cols = columns(es.P, X, Y, nrm, alpha, R, t)
            nll = es.nll
        else:
            cols, nll = estep_columns(R, t, s2)
        out.nll.append(nll)
        if tol > 0 and prev is not None and abs(nll - prev) <= tol * abs(nll):
            break
        prev = nll
        ms = mstep(cols, X, R, t, s2, newton_max=newton_max, sigma2_floor=floor)
        R, t, s2 = ms.R, ms.t, ms.sigma2
        out.gn_fallbacks += ms.gn_fallbacks
        out.iters = it + 1
        out.sigma2_trace.append(s2)
        out.R_trace.append(R.copy())
        out.t_trace.append(t.copy())
    out.R, out.t, out.sigma2 = R, t, s2
    return out


# ----------------------------------------------------------------------------
# Evaluation (Sec. 4)
# ----------------------------------------------------------------------------

def registration_error(X, R, t, R_gt, t_gt):
    """Eq. (14): mean distance between g(x_i) and g_gt(x_i)."""
    X = _f64(X)
    d = X @ (_f64(R) - _f64(R_gt)).T + (_f64(t) - _f64(t_gt))
    return float(np.mean(np.sqrt(np.sum(d * d, axis=1))))


def rotation_error_deg(R, R_gt):
    """Angle of the axis-angle form of R_gt^T R (Sec. 4.4), in degrees,
    evaluated with atan2 so that it stays accurate near zero."""
    dR = _f64(R_gt).T @ _f64(R)
    s = 0.5 * np.linalg.norm([dR[2, 1] - dR[1, 2], dR[0, 2] - dR[2, 0], dR[1, 0] - dR[0, 1]])
    c = 0.5 * (np.trace(dR) - 1.0)
    return math.degrees(math.atan2(s, c))


def translation_error(t, t_gt):
    """Euclidean distance between translations (Sec. 4.4)."""
    return float(np.linalg.norm(_f64(t) - _f64(t_gt)))
