"""Writes the stored expected values under tests/golden/ from the FP64 oracle
only (no GPU code is imported).  Run: python tests/golden/make_golden.py

* alpha_eq3.json      -- the penalty of Eq. 3 on a grid of surface variations
* estep_small.json    -- one E step (Eq. 5 in the form of Eq. 9) of a 12 x 9
                         pair: inputs (float32 values), P, NLL (Eq. 4)
* register_small.json -- 30 EM iterations (Sec. 3) of a 300 x 250 pair: the
                         final pose, sigma^2 and the NLL per iteration
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import datagen  # noqa: E402
from oracle import lsgcpd_oracle as O  # noqa: E402


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64).tolist()


def alpha_case():
    kappa = [0.0, 1e-4, 0.01, 0.05, 0.1, 0.2, 0.3, 1.0 / 3.0]
    return {"source": "Eq. 3 (penalty alpha from the surface variation kappa)",
            "alpha_max": 30.0, "lambda": 0.2, "kappa": kappa,
            "alpha": O.penalty_alpha(np.array(kappa), 30.0, 0.2).tolist()}


def estep_case():
    p = datagen.range_scanner_pair(trial=11, M=12, N=9)
    n, _, a = O.normals(p.Y, 5, 30.0, 0.2)
    n32, a32 = n.astype(np.float32), a.astype(np.float32)
    rng = np.random.default_rng(11)
    R = datagen.random_rotation(rng, 0.2)
    t = rng.normal(size=3) * 0.05
    s2, w0, V = 0.02, 0.1, 2.0
    es = O.estep(p.X, p.Y, n32, a32, R, t, s2, w0=w0, V=V)
    return {"source": "Eq. 5 in the form of Eq. 9 with Eq. 2's component density; NLL of Eq. 4",
            "X": f32(p.X), "Y": f32(p.Y), "normals": f32(n32), "alpha": f32(a32),
            "R": R.tolist(), "t": t.tolist(), "sigma2": s2, "w0": w0, "V": V,
            "P": es.P.tolist(), "nll": es.nll, "gamma": es.gamma}


def register_case():
    p = datagen.range_scanner_pair(trial=12, M=300, N=250, angle_deg=20.0)
    r = O.register(p.X, p.Y, k=10, max_iter=30)
    return {"source": "Sec. 3: normals (Eq. 3), EM with the E step of Eq. 9 and the Newton "
                      "M step on SE(3) (Eq. 11-13), sigma^2 update of Sec. 3.5",
            "X": f32(p.X), "Y": f32(p.Y), "k": 10, "max_iter": 30, "w0": 0.1,
            "alpha_max": 30.0, "lambda": 0.2,
            "R": r.R.tolist(), "t": r.t.tolist(), "sigma2": r.sigma2, "nll": list(r.nll),
            "iters": r.iters}


def main():
    for name, fn in (("alpha_eq3.json", alpha_case), ("estep_small.json", estep_case),
                     ("register_small.json", register_case)):
        rec = fn()
        rec["written_by"] = "tests/golden/make_golden.py (oracle only)"
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(rec, f, indent=1)
        print("wrote", name)


if __name__ == "__main__":
    main()
